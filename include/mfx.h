/*
 * mfx — finite-volume right-hand side and SSP-RK3 step of the two-component
 * five-equation diffuse-interface model on one MI355X (gfx950).
 *
 * Method (arXiv 2409.10729, "OpenACC offloading of the MFC compressible
 * multiphase flow solver on AMD and NVIDIA GPUs"):
 *   Sec. II-A  Allaire five-equation model, stiffened-gas EOS with mixture
 *              parameters;
 *   Sec. II-B  eq. (discretization) and its cell-integrated form (eq. rhs):
 *              dq/dt = sum_d (F_{-1/2} - F_{+1/2}) / dx_d - h(q) div(u),
 *              HLLC fluxes from WENO5 face states.
 * Readings of what the paper leaves open (mixture rules, reconstructed
 * variables, WENO epsilon, wave speeds, time integrator, CFL rule, boundary
 * conditions) are fixed as documented for each call below.
 *
 * Data layout (every call): conserved state q is float64, structure of
 * arrays, q[v][k][j][i] with x (i) fastest, no ghost cells, v =
 *   0 alpha1*rho1, 1 alpha2*rho2, 2 rho*u, 3 rho*v, 4 rho*w, 5 rho*E, 6 alpha1.
 * Primitive layout (mfx_set_primitive) is the same with (u, v, w, p) in
 * slots 2..5.  All pointers named *_dev are device pointers on the device
 * current when mfx_init_grid was called.
 *
 * Ownership: the caller owns the workspace and every state buffer; the
 * library owns only the host-side context.  The workspace must stay
 * allocated until mfx_destroy.  Calls are enqueued on the stream given to
 * mfx_init_grid and are asynchronous unless stated; a context is bound to
 * one stream and is not thread-safe.
 *
 * Errors: every int-returning call returns MFX_OK (0) or a negative code;
 * the message is available from mfx_last_error.  Bad arguments are
 * reported synchronously (MFX_EINVAL) before anything is enqueued.
 * Non-physical states seen by a kernel (rho <= 0, non-positive squared
 * sound speed, non-finite values) raise a device status bit that the next
 * synchronising call (mfx_stats, mfx_get_state, mfx_rk3_step with a host
 * dt readback) returns as MFX_ESTATE.  No C++ exception crosses the ABI.
 */
#ifndef MFX_H
#define MFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MFX_OK = 0,
    MFX_EINVAL = -1, /* invalid argument or descriptor */
    MFX_EHIP = -2,   /* a HIP runtime call failed */
    MFX_ENOMEM = -3, /* workspace smaller than mfx_workspace_bytes */
    MFX_ESTATE = -4  /* non-physical or non-finite state detected on the device */
};

enum { MFX_BC_PERIODIC = 0, MFX_BC_TRANSMISSIVE = 1 };

/* Arithmetic of the reconstruction and flux passes.
 * MFX_FP64: everything in float64.
 * MFX_FP32_MIXED: WENO, HLLC and flux divergence in float32; the pressure
 *   inversion of every cell, the RK stage accumulation of the conserved
 *   state and the CFL reduction stay float64; the stored RHS is float32. */
enum { MFX_FP64 = 0, MFX_FP32_MIXED = 1 };

/* Nonlinear WENO weights.  MFX_WENO5_JS: Jiang-Shu.  MFX_WENO5_LEARNED: a
 * 5-32-32-3 MLP (set with mfx_set_mlp) maps scale-free smoothness features
 * to the three weights, with Jiang-Shu as the fallback wherever the learned
 * weights leave the convex set or the face state fails a positivity check. */
enum { MFX_WENO5_JS = 0, MFX_WENO5_LEARNED = 1 };

typedef struct {
    int32_t n[3];      /* interior cells (nx, ny, nz), each >= 1; n == 1 makes a direction inactive */
    double lo[3];      /* domain origin (informational) */
    double dx[3];      /* uniform spacing per direction, > 0 */
    int32_t bc[3][2];  /* lower/upper boundary per direction; periodic must be paired */
    double gamma[2];   /* stiffened-gas gamma of fluid 1 and fluid 2, > 1 */
    double pi_inf[2];  /* stiffened-gas pi_inf of fluid 1 and fluid 2, >= 0 */
    double cfl;        /* CFL number for the automatic time step, in (0, 1] */
    double weno_eps;   /* WENO epsilon (absolute), > 0; 1e-6 is Jiang-Shu's value */
    int32_t precision; /* MFX_FP64 or MFX_FP32_MIXED */
    int32_t weights;   /* MFX_WENO5_JS or MFX_WENO5_LEARNED */
} mfx_grid_desc;

typedef struct mfx_ctx mfx_ctx;

/* Bytes of device workspace a context needs for this descriptor (three
 * state-sized float64 buffers, one RHS buffer and small reduction space).
 * Returns 0 for an invalid descriptor.  Host-only; touches no device. */
size_t mfx_workspace_bytes(const mfx_grid_desc* desc);

/* Validate the descriptor (Sec. II-A/II-B parameters above) and bind a
 * context to the caller's workspace (device pointer, >= mfx_workspace_bytes)
 * and HIP stream (hipStream_t passed as void*, NULL = default stream).
 * On success *out receives the context.  The state is undefined until
 * mfx_set_state or mfx_set_primitive. */
int mfx_init_grid(const mfx_grid_desc* desc, void* ws_dev, size_t ws_bytes, void* hip_stream,
                  mfx_ctx** out);

/* Copy a conserved state (layout above) into the context and compute its
 * CFL time step on the device.  The caller's buffer may be reused as soon
 * as the call returns only after the stream has reached this point. */
int mfx_set_state(mfx_ctx* ctx, const double* q_dev);

/* Same, from primitive variables (alpha1 rho1, alpha2 rho2, u, v, w, p,
 * alpha1); the conversion uses the mixture stiffened-gas EOS of Sec. II-A:
 * rho E = Gamma(alpha1) p + Pi(alpha1) + rho |u|^2 / 2 with
 * Gamma = sum_i alpha_i / (gamma_i - 1), Pi = sum_i alpha_i gamma_i pi_i / (gamma_i - 1). */
int mfx_set_primitive(mfx_ctx* ctx, const double* w_dev);

/* Copy the current conserved state out (same layout).  Synchronises the
 * stream; returns MFX_ESTATE if a kernel flagged a non-physical state. */
int mfx_get_state(mfx_ctx* ctx, double* q_dev_out);

/* Right-hand side L(q) of eq. (rhs) for the current state: for each active
 * direction in the order x, y, z, WENO5 face states of the primitive
 * variables, HLLC fluxes and face velocities, flux differences over dx, and
 * the alpha1 source alpha1 (u_f,+1/2 - u_f,-1/2) / dx.  Ghost cells come
 * from the boundary conditions (periodic wrap; transmissive = zero-gradient
 * copy of the boundary cell).  Written as float64 in the state layout to
 * rhs_dev_out (which must not alias the workspace).  Asynchronous. */
int mfx_rhs(mfx_ctx* ctx, double* rhs_dev_out);

/* One SSP-RK3 step (Shu-Osher form) of the current state:
 *   q1 = q + dt L(q);  q2 = 3/4 q + 1/4 (q1 + dt L(q1));
 *   q  = 1/3 q + 2/3 (q2 + dt L(q2)).
 * dt > 0 uses that time step.  dt <= 0 uses the CFL time step of the
 * current state, dt = cfl / max over cells of sum_d (|u_d| + c) / dx_d,
 * which stays on the device (no synchronisation); a grid with no active
 * direction (1x1x1) has no CFL time step and needs dt > 0 (else MFX_EINVAL).  If dt_used_host is not
 * NULL the call synchronises and stores the time step used there (and
 * reports MFX_ESTATE if a kernel flagged a state).  The CFL time step of
 * the new state is computed inside the step for the next call. */
int mfx_rk3_step(mfx_ctx* ctx, double dt, double* dt_used_host);

/* Learned-weight parameters: n_params float32 values on the device, laid
 * out W1[32][5], b1[32], W2[32][32], b2[32], W3[3][32], b3[3] (1347 values).
 * Copied and packed to bfloat16 for inference. */
int mfx_set_mlp(mfx_ctx* ctx, const float* params_dev, int32_t n_params);

/* Synchronise and report simulated time, step count, faces that fell back
 * to Jiang-Shu weights (learned mode), and the device status word.  Any
 * pointer may be NULL.  Returns MFX_ESTATE if the status word is non-zero. */
int mfx_stats(mfx_ctx* ctx, double* t, int64_t* step, int64_t* fallback_faces, uint32_t* status);

/* Kernel timing for measurement.  mfx_profile(ctx, 1) clears the counters
 * and brackets every sweep launch with HIP events on the context's stream
 * (0 stops).  mfx_profile_read synchronises and returns, per launch kind,
 * the summed event time in milliseconds and the launch count since the
 * last mfx_profile call; kind = (direction * 2 + first_pass) * 5 + output,
 * output 0 partial RHS, 1 caller RHS, 2/3/4 RK stage 1/2/3.  Arrays hold
 * MFX_PROF_KINDS entries; either may be NULL. */
#define MFX_PROF_KINDS 30
int mfx_profile(mfx_ctx* ctx, int enable);
int mfx_profile_read(mfx_ctx* ctx, double* ms, int64_t* counts);

/* Release the host-side context (the workspace stays the caller's). */
void mfx_destroy(mfx_ctx* ctx);

/* Message of the last error on this context (or of the last failed
 * mfx_init_grid when ctx is NULL). */
const char* mfx_last_error(const mfx_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MFX_H */
