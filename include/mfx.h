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
 * arrays, q[v][k][j][i] with x (i) fastest, no ghost cells; two fluids:
 *   0 alpha1*rho1, 1 alpha2*rho2, 2 rho*u, 3 rho*v, 4 rho*w, 5 rho*E, 6 alpha1;
 * nf fluids (mfx_grid_desc.num_fluids): alpha_i rho_i (i = 1..nf), rho u,
 * rho v, rho w, rho E, alpha_1 .. alpha_{nf-1}, 2 nf + 3 variables.
 * Primitive layout (mfx_set_primitive) is the same with (u, v, w, p) in
 * place of momentum and energy.  All pointers named *_dev are device pointers on the device
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
 * Non-physical states seen by a kernel raise bits of a device status word
 * (MFX_STATUS_* below); an error bit is returned as MFX_ESTATE by the next
 * synchronising call (mfx_stats, mfx_get_state, mfx_rk3_step with a host
 * dt readback).  No C++ exception crosses the ABI.
 */
#ifndef MFX_H
#define MFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status word bits.  The state a call sets (mfx_set_state,
 * mfx_set_primitive) and the new state of every step are checked for all
 * four; the intermediate RK stages for the first three when their last pass
 * is a y or z sweep (3D grids and grids with z active).  MFX_STATUS_ALPHA
 * is recorded but is not an error: the unlimited scheme (no clipping) can
 * carry alpha1 slightly outside [0, 1] next to a sharp interface (about
 * 1e-6 below 0 and 2e-4 above 1 in the water/air shock tube), and such a
 * state stays computable. */
#define MFX_STATUS_RHO 1u        /* density alpha1 rho1 + alpha2 rho2 not positive */
#define MFX_STATUS_SOUND 2u      /* squared sound speed ((Gamma+1) p + Pi)/(Gamma rho) not positive */
#define MFX_STATUS_NONFINITE 4u  /* a non-finite value */
#define MFX_STATUS_ALPHA 8u      /* alpha1 outside [0, 1] (recorded, not an error) */
#define MFX_STATUS_ERRORS (MFX_STATUS_RHO | MFX_STATUS_SOUND | MFX_STATUS_NONFINITE)

enum {
    MFX_OK = 0,
    MFX_EINVAL = -1, /* invalid argument or descriptor */
    MFX_EHIP = -2,   /* a HIP runtime call failed */
    MFX_ENOMEM = -3, /* workspace smaller than mfx_workspace_bytes */
    MFX_ESTATE = -4  /* non-physical or non-finite state detected on the device */
};

/* Boundary types (ghost cells, Sec. III-A structured mesh; the paper names
 * none, these are the standard constructions).  Periodic wraps around and
 * must be paired; transmissive repeats the edge cell (zero gradient);
 * reflective is a stationary slip wall: the ghost cells mirror the cells
 * beside the wall face with the momentum normal to it negated, so no mass
 * or energy crosses it; it needs at least 3 cells in its direction.
 * Inflow: every ghost cell of the side holds the fixed conserved state
 * mfx_grid_desc.inflow[direction][side]. */
enum { MFX_BC_PERIODIC = 0, MFX_BC_TRANSMISSIVE = 1, MFX_BC_REFLECTIVE = 2, MFX_BC_INFLOW = 3 };

/* Arithmetic of the reconstruction and flux passes.
 * MFX_FP64: everything in float64.
 * MFX_FP32_MIXED: WENO, HLLC and flux divergence in float32; the pressure
 *   inversion of every cell, the RK stage accumulation of the conserved
 *   state and the CFL reduction stay float64; the stored RHS is float32. */
enum { MFX_FP64 = 0, MFX_FP32_MIXED = 1 };

/* Nonlinear WENO weights.  MFX_WENO5_JS: Jiang-Shu.  MFX_WENO5_LEARNED: a
 * 5-32-32-3 MLP (set with mfx_set_mlp) maps scale-free smoothness features
 * to the three weights, with Jiang-Shu as the fallback wherever the learned
 * weights leave the convex set or the face state fails a positivity check;
 * one evaluation per variable and edge.  MFX_WENO5_LEARNED_EDGE: the same
 * network evaluated once per edge for all seven variables, on the
 * componentwise maximum of the variables' features; its logits correct each
 * variable's own Jiang-Shu weights; same fallback.  Both learned modes run in the MFX_FP32_MIXED form.
 * MFX_WENO5_Z: WENO-Z weights (Borges, Carmona, Costa & Don 2008, exponent
 * 1), alpha_k = d_k (1 + |beta_0 - beta_2| / (beta_k + eps)), a comparison
 * form for the learned weights; any precision form. */
enum { MFX_WENO5_JS = 0, MFX_WENO5_LEARNED = 1, MFX_WENO5_LEARNED_EDGE = 2, MFX_WENO5_Z = 3 };

/* Fluids the library takes (num_fluids), and the variables of the largest
 * model (2 * fluids + 3). */
#define MFX_MAX_FLUIDS 3
#define MFX_MAX_VARS (2 * MFX_MAX_FLUIDS + 3)

typedef struct {
    int32_t n[3];      /* interior cells (nx, ny, nz), each >= 1; n == 1 makes a direction inactive */
    double lo[3];      /* domain origin (informational) */
    double dx[3];      /* uniform spacing per direction, > 0 */
    int32_t bc[3][2];  /* lower/upper MFX_BC_* per direction; periodic must be paired */
    double gamma[MFX_MAX_FLUIDS];  /* stiffened-gas gamma of each fluid, > 1 (the first num_fluids used) */
    double pi_inf[MFX_MAX_FLUIDS]; /* stiffened-gas pi_inf of each fluid, >= 0 */
    double cfl;        /* CFL number for the automatic time step, in (0, 1] */
    double weno_eps;   /* WENO epsilon (absolute), > 0; 1e-6 is Jiang-Shu's value */
    int32_t precision; /* MFX_FP64 or MFX_FP32_MIXED */
    int32_t weights;   /* MFX_WENO5_JS, MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE or MFX_WENO5_Z */
    int32_t weno_order; /* reconstruction order, 5 or 3 (Sec. II-B names both; 0 reads as 5):
                           WENO3 with Jiang-Shu weights on the middle three cells of each
                           stencil; the learned and WENO-Z weights need 5 (MFX_EINVAL otherwise) */
    double inflow[3][2][MFX_MAX_VARS]; /* conserved ghost state (the first 2 num_fluids + 3 entries,
                               in the state layout) of each MFX_BC_INFLOW side [direction][lower/upper];
                               finite, partial densities >= 0 with a positive sum, volume fractions
                               in [0, 1] summing to at most 1 (MFX_EINVAL otherwise); ignored for
                               other sides */
    int32_t num_fluids; /* fluids of the model, 2 .. MFX_MAX_FLUIDS (0 reads as 2).  Sec. II-A
                           states the system for two components with a continuity and a
                           volume-fraction equation per component; with nf components the state
                           holds nf partial densities, the momentum, the energy and the volume
                           fractions alpha_1 .. alpha_{nf-1} (alpha_nf = 1 - their sum), the mixture
                           rules stay linear in every fraction and every fraction carries its
                           alpha_i div(u) source.  More than two fluids: Jiang-Shu-family
                           weights (the learned weights are for two) */
    const double* faces[3]; /* unequal cell widths along a direction (Sec. III-A: a structured mesh
                           refined locally, e.g. by hyperbolic-tangent stretching): a HOST pointer
                           to the n[d] + 1 face coordinates of direction d, finite and strictly
                           increasing, or NULL for uniform cells of width dx[d] (dx[d] is then
                           ignored).  Read only by mfx_workspace_bytes and mfx_init_grid, which
                           derive per-cell WENO5 coefficient tables from the widths (the caller may
                           free the array afterwards); the direction must be active (n[d] > 1) and
                           the reconstruction WENO5 with Jiang-Shu weights (weno_order 5,
                           MFX_WENO5_JS).  A ghost cell takes the width of the cell whose state the
                           boundary rule gives it.  mfx_rhs_static takes uniform grids only */
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
 * mfx_set_state or mfx_set_primitive.
 * Kernel-choice switches read from the environment here (and by
 * mfx_workspace_bytes), for testing the equivalent paths against each
 * other; results agree to rounding either way:
 *   MFX_FUSE_XY=0    separate x and y passes instead of the fused x-y pass;
 *   MFX_FUSE_CFL=0   the CFL reduction as its own pass after each step
 *                    instead of inside the step's last y/z pass;
 *   MFX_XSWEEP=march the marching x pass instead of whole rows;
 *   MFX_SWEEP_SEG=n  segment length of the marching passes (default 64). */
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
 * stream; returns MFX_ESTATE if a kernel set an error bit of the status
 * word. */
int mfx_get_state(mfx_ctx* ctx, double* q_dev_out);

/* Right-hand side L(q) of eq. (rhs) for the current state: for each active
 * direction in the order x, y, z, WENO face states of the primitive
 * variables (the descriptor's order and weights), HLLC fluxes and face
 * velocities, flux differences over dx, and the alpha1 source
 * alpha1 (u_f,+1/2 - u_f,-1/2) / dx.  Ghost cells come from the boundary
 * conditions (MFX_BC_*: periodic wrap, transmissive zero-gradient copy,
 * reflective mirror with the normal momentum negated, inflow fixed state).
 * Written as float64 in the state layout to rhs_dev_out (which must not
 * alias the workspace).  Asynchronous.  The state was checked when it was
 * set or stepped (status word); this call checks nothing further. */
int mfx_rhs(mfx_ctx* ctx, double* rhs_dev_out);

/* One SSP-RK3 step (Shu-Osher form) of the current state:
 *   q1 = q + dt L(q);  q2 = 3/4 q + 1/4 (q1 + dt L(q1));
 *   q  = 1/3 q + 2/3 (q2 + dt L(q2)).
 * dt > 0 uses that time step.  dt <= 0 uses the CFL time step of the
 * current state, dt = cfl / max over cells of sum_d (|u_d| + c) / dx_d,
 * which stays on the device (no synchronisation); a grid with no active
 * direction (1x1x1) has no CFL time step and needs dt > 0 (else MFX_EINVAL).  If dt_used_host is not
 * NULL the call synchronises and stores the time step used there (and
 * returns MFX_ESTATE if an error bit of the status word is set).  The CFL time step of
 * the new state is computed inside the step for the next call. */
int mfx_rk3_step(mfx_ctx* ctx, double dt, double* dt_used_host);

/* Learned-weight parameters: n_params (= 1347) float32 values on the
 * device, laid out W1[32][5], b1[32], W2[32][32], b2[32], W3[3][32], b3[3].
 * Copied into the context and packed to bfloat16 for the matrix cores.
 * Needed before the first step of a context created with a learned
 * weights mode (which runs in the MFX_FP32_MIXED precision form).  In
 * that form every cell's two edge states come from the network's weights,
 * and an edge whose weights are not finite or whose state is not admissible
 * (negative partial density, alpha1 outside [0,1], non-positive squared
 * sound speed) falls back to Jiang-Shu for all seven variables; mfx_stats
 * counts those edges.  A variable whose 5-cell stencil is constant on all
 * 64 cells a wavefront handles takes the Jiang-Shu edge values without
 * evaluating the network (any convex weights give the constant).  The
 * parameters may be replaced between steps; the call is ordered on the
 * context's stream. */
int mfx_set_mlp(mfx_ctx* ctx, const float* params_dev, int32_t n_params);

/* Synchronise and report simulated time, step count, faces that fell back
 * to Jiang-Shu weights (learned mode), and the device status word
 * (MFX_STATUS_* bits, accumulated since the state was set).  Any pointer
 * may be NULL.  Returns MFX_ESTATE if an error bit (MFX_STATUS_ERRORS) is
 * set. */
int mfx_stats(mfx_ctx* ctx, double* t, int64_t* step, int64_t* fallback_faces, uint32_t* status);

/* ------------------------------------------------------------------------
 * Learned WENO weights: training and stand-alone inference.
 *
 * The network maps five features of a 5-cell stencil w0..w4 reconstructed
 * at its right edge -- with the Jiang-Shu indicators beta_k (Shu 2006, the
 * WENO5 of Sec. II-B) and S = beta0 + beta1 + beta2 + eps:
 *   (beta0/S, beta1/S, beta2/S, |beta0 - beta2|/S, D^2/(S + D^2)),
 *   D = w0 - 4 w1 + 6 w2 - 4 w3 + w4
 * -- through 5 -> 32 (GELU) -> 32 (GELU) -> 3 logits z, which correct the
 * Jiang-Shu weights of the third-order candidates:
 *   omega = softmax(ln omega_JS + z)
 * (a zero output layer reproduces Jiang-Shu exactly).  GELU is trained in
 * its tanh form, a (1 + tanh(sqrt(2/pi) (a + 0.044715 a^3))) / 2, and
 * evaluated at inference as max(a, 0) - t Q(t), t = min(|a|, 3.75), with Q
 * a degree-6 minimax fit of the tanh form's remainder (within 1.2e-4 of the
 * tanh form; the inference operands are bfloat16).  Parameters: 1347
 * float32, layout of mfx_set_mlp.  A left edge is the right edge of the
 * mirrored stencil.  These calls are not bound to a context; all pointers
 * are device pointers, work is enqueued on `stream` (hipStream_t as void*,
 * NULL = default stream), and errors are returned as codes with the message
 * in mfx_mlp_last_error().
 * ---------------------------------------------------------------------- */
#define MFX_MLP_PARAMS 1347

/* Training samples from a 1D state q[7][nx] (desc->n = {nx,1,1}; its x
 * boundary conditions give the ghost cells).  For every cell i and variable
 * v two samples are written: sample (0*7+v)*nx+i = primitives w[v] of cells
 * i-2..i+2 with target face_prim[v][i+1]; sample (1*7+v)*nx+i = the
 * mirrored stencil i+2..i-2 with target face_prim[v][i].  face_prim holds
 * reference primitive values at the nx+1 faces, [7][nx+1].  Outputs:
 * stencil_out[14*nx][5], target_out[14*nx] (float64).  Reflective and inflow
 * ends are rejected (MFX_EINVAL). */
int mfx_mlp_sample_stencils(const mfx_grid_desc* desc, const double* q_dev, const double* face_prim_dev,
                            double* stencil_out, double* target_out, void* stream);

/* Reference face values for training targets from a 1D state on a grid
 * `refine` times finer than the sampled one (same domain and boundary
 * conditions): coarse face i lies on fine face refine*i, whose primitive
 * value is the mean of the two fine cells beside it.  face_prim_out[7][nc+1]
 * with nc = fine nx / refine.  Reflective and inflow ends are rejected
 * (MFX_EINVAL). */
int mfx_mlp_face_targets(const mfx_grid_desc* fine_desc, const double* q_fine_dev, int32_t refine, double* face_prim_out,
                         void* stream);

/* Features (float32 [n][5]), Jiang-Shu weights (omega_js [n][3]) and the
 * stencil-normalised candidates cand[n][3] and target tnorm[n] of n
 * samples: (x - w2) / (max - min of the stencil), zero for a flat stencil. */
int mfx_mlp_features(const double* stencils, const double* targets, int64_t n, double eps, float* feat, float* cand,
                     float* tnorm, float* omega_js, void* stream);

/* Shared (per-edge) form: samples of a 1D sample set as
 * mfx_mlp_sample_stencils lays it out (stencils [14*ncell][5], targets
 * [14*ncell]).  Sample j = side*ncell + i (j < 2*ncell) gets feat[j][5] =
 * componentwise maximum over the seven variables of their features, and per
 * variable omega_base[j][7][3] = its Jiang-Shu weights, cand[j][7][3],
 * tnorm[j][7] normalised as in mfx_mlp_features; a variable with a flat
 * stencil or with |tnorm| > tmax contributes zero candidates and target. */
int mfx_mlp_features_edge(const double* stencils, const double* targets, int64_t ncell, double eps, double tmax,
                          float* feat, float* cand, float* tnorm, float* omega_base, void* stream);

/* Bytes of the packed bfloat16 matrix-core operands (mfx_mlp_pack). */
size_t mfx_mlp_packed_bytes(void);
/* Pack float32 parameters into the matrix-core operand words: for each of
 * the 64 lanes of a wave, its bfloat16 A-operand fragments of the three
 * layers and its float32 bias registers, stored word-major (word w of
 * every lane contiguous) so that a wave reads each word as one contiguous
 * kilobyte. */
int mfx_mlp_pack(const float* params, void* packed, void* stream);

/* Network weights omega[n][3] for features feat[n][5] and Jiang-Shu
 * weights omega_js[n][3]: pass params (float32 arithmetic) or packed
 * (bfloat16 matrix cores, float32 accumulation, as inside the solver), not
 * both. */
int mfx_mlp_forward(const float* params, const void* packed, const float* feat, const float* omega_js, int64_t n,
                    float* omega, void* stream);

/* Loss and gradient of one minibatch, float32, deterministic (per-block
 * sums in a fixed order, then a fixed-order sum over blocks), with nvar
 * (1, or 7 for the shared form) variables per sample sharing its logits z,
 * each correcting its own baseline: omega_iv = softmax(ln omega_js_iv + z_i),
 *   L = mean_i (1/nvar) sum_v [ (sum_k omega_ivk cand_ivk - tnorm_iv)^2
 *                               + lambda sum_k (omega_ivk - omega_js_ivk)^2 ],
 * cand and omega_js [n][nvar][3], tnorm[n][nvar].  grad_out[1347]; loss_out (device
 * float, may be NULL); ws of at least mfx_mlp_grad_workspace(n) bytes. */
size_t mfx_mlp_grad_workspace(int64_t n);
int mfx_mlp_loss_grad(const float* params, const float* feat, const float* cand, const float* tnorm,
                      const float* omega_js, int64_t n, int32_t nvar, float lambda, void* ws, size_t ws_bytes,
                      float* grad_out, float* loss_out, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) of the parameters with
 * first/second moment buffers m, v (1347 each); step counts from 1. */
int mfx_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step, float lr, void* stream);

/* Message of the last failed learned-weights call of this thread. */
const char* mfx_mlp_last_error(void);

/* Kernel timing for measurement.  mfx_profile(ctx, 1) clears the counters
 * and brackets every sweep launch with HIP events on the context's stream
 * (0 stops).  mfx_profile_read synchronises and returns, per launch kind,
 * the summed event time in milliseconds and the launch count since the
 * last mfx_profile call; kind = (direction * 2 + first_pass) * 5 + output,
 * output 0 partial RHS, 1 caller RHS, 2/3/4 RK stage 1/2/3; direction 3
 * is the fused x-y pass (x and y in one kernel, used when both are active
 * with equal cells, an x row fits the row kernel (nx <= 512), the weights
 * are Jiang-Shu-family and the model is not three fluids in float64;
 * MFX_FUSE_XY=0 in the environment at mfx_init_grid turns it off).  Arrays hold MFX_PROF_KINDS entries;
 * either may be NULL. */
#define MFX_PROF_KINDS 40
int mfx_profile(mfx_ctx* ctx, int enable);
int mfx_profile_read(mfx_ctx* ctx, double* ms, int64_t* counts);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * right-hand side of mfx_rhs for the state q_dev (layout above) on the
 * descriptor's grid, with no context and no workspace.  Its scratch (the
 * partial right-hand side, the x rows' boundary faces, the inflow states)
 * lives in a static device array of MFX_STATIC_SCRATCH_BYTES that every GPU
 * the library runs on holds until the process ends; the call allocates
 * nothing.  Scratch a grid needs: 768 + a(e * 2 (nv + 1) * ny * nz) + a(e * nv *
 * nx * ny * nz) bytes, a() rounding up to a multiple of 256, e = 8 for MFX_FP64
 * and 4 for MFX_FP32_MIXED, nv = 2 num_fluids + 3 (two fluids: up to about
 * 2.3 million cells in float64, e.g. 128^3, and 4.6 million in float32); a
 * larger grid is rejected with MFX_ENOMEM before anything is enqueued.  Jiang-Shu or WENO-Z weights,
 * order 5 or 3 (learned weights need a context: MFX_EINVAL), uniform cells
 * (mfx_grid_desc.faces all NULL, else MFX_EINVAL).  q_dev and
 * rhs_dev_out are device pointers on the current device and must not
 * overlap.  Enqueued on hip_stream (hipStream_t as void*, NULL = default
 * stream); asynchronous.  Every call on one GPU uses that GPU's one array,
 * which keeps the last call's contents (nothing in it is read before the
 * call writes it): calls that overlap in time on one GPU (other streams,
 * other threads) race, and the caller must order them.  Errors are returned
 * as codes with the message in mfx_last_error(NULL). */
#define MFX_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
int mfx_rhs_static(const mfx_grid_desc* desc, const double* q_dev, double* rhs_dev_out, void* hip_stream);

/* WENO5 coefficients on cells of unequal widths (Sec. III-A local mesh
 * refinement; Sec. II-B's WENO5 on the refined mesh), as the library derives
 * them for every stencil position of a direction given by
 * mfx_grid_desc.faces.  h: the widths of the five cells c-2 .. c+2 (host
 * array, finite and > 0).  out (host array of MFX_NU_COEFS doubles):
 *   out[ 0.. 8] a[k][i], out[ 9..17] b[k][i], out[18..26] c[k][i]: candidate
 *     k (cells c-2+k .. c+k) is A_k + B_k xi + C_k xi^2 in the middle cell's
 *     coordinate xi = (x - x_c) / h_c, with A_k = sum_i a[k][i] v_{c-2+k+i}
 *     (likewise B, C) for cell averages v;
 *   out[27..29] ideal weights of the right edge (xi = 1/2), out[30..32]
 *     those of the left edge (xi = -1/2).
 * Smoothness indicator beta_k = B_k^2 + 13/3 C_k^2.  Host-only (touches no
 * device); MFX_EINVAL for a NULL pointer or a width that is not finite and
 * positive. */
#define MFX_NU_COEFS 33
int mfx_weno5_nu_coefficients(const double* h, double* out);

/* Release the host-side context (the workspace stays the caller's). */
void mfx_destroy(mfx_ctx* ctx);

/* Message of the last error on this context (or of the last failed
 * mfx_init_grid when ctx is NULL). */
const char* mfx_last_error(const mfx_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MFX_H */
