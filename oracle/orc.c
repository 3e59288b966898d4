/*
 * Plain FP64 CPU oracle for the finite-volume right-hand side of the
 * two-component five-equation (Allaire) diffuse-interface model and its
 * SSP-RK3 time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU library; both sides only read
 * the same seeded input arrays.
 *
 * What it follows (paper: "OpenACC offloading of the MFC compressible
 * multiphase flow solver on AMD and NVIDIA GPUs", arXiv 2409.10729):
 *   - model:      Sec. II-A, the two-component Allaire system (the
 *                 unnumbered align block), read as partial-density
 *                 continuity, mixture momentum and energy, and alpha_1
 *                 advection;
 *   - EOS:        Sec. II-A, stiffened gas with mixture gamma, pi_inf
 *                 (mixture rules linear in alpha_1 for 1/(gamma-1) and
 *                 gamma*pi_inf/(gamma-1), after Allaire et al. 2002);
 *   - scheme:     Sec. II-B, eq. (discretization) and the cell-integrated
 *                 form below it (eq. rhs): flux differences per direction
 *                 minus h(q) div(u), with HLLC fluxes (Toro 2009) from
 *                 WENO5 face states (Shu 2006, Jiang-Shu weights);
 *   - h(q):       only the alpha_1 equation carries a source, +alpha_1
 *                 div(u), with div(u) built from the HLLC face velocity
 *                 (Johnsen & Colonius 2006, the approach the cited
 *                 Coralic-Colonius scheme uses);
 *   - time:       SSP-RK3 in Shu-Osher form, CFL time step from the sum
 *                 over directions of (|u_d| + c) / dx_d.
 *
 * Conserved variables, in this order, stored structure-of-arrays as
 * q[v][k][j][i] (x fastest):
 *   0: alpha1*rho1  1: alpha2*rho2  2: rho*u  3: rho*v  4: rho*w
 *   5: rho*E        6: alpha1
 * Primitive variables (same order): alpha1*rho1, alpha2*rho2, u, v, w, p,
 * alpha1.
 *
 * Ghost cells are materialised in a padded copy (3 layers per active
 * direction) filled by periodic wrap or zero-gradient copy.  Built with
 * -O2 -fno-fast-math -ffp-contract=off; OpenMP over pencils only, so the
 * result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 7 /* variables of the two-fluid model (the learned weights) */
#define NG 3
#define NFMAX 4 /* fluids */
#define NVMAX (2 * NFMAX + 3)

typedef struct {
    int32_t n[3];      /* interior cells per direction; 1 = inactive */
    double dx[3];      /* uniform spacing per direction */
    int32_t bc[3][2];  /* 0 = periodic, 1 = transmissive (zero gradient),
                          2 = reflective (slip wall), 3 = inflow (fixed state) */
    double gamma[NFMAX]; /* per fluid */
    double pinf[NFMAX];
    double eps;        /* WENO epsilon */
    double cfl;
    int32_t weno_z;    /* 0: Jiang-Shu weights (the paper's WENO5); 1: WENO-Z weights (comparison form) */
    int32_t weno_order; /* 5 (default; 0 reads as 5) or 3: the two orders Sec. II-B names */
    double inflow[3][2][NVMAX]; /* conserved state of the ghost cells of an inflow side */
    int32_t nf;        /* fluids, 2..NFMAX (0 reads as 2) */
    const double* xf[3]; /* face coordinates of a non-uniform direction (n + 1, increasing),
                            or NULL for uniform cells of width dx */
} orc_grid;

/* Variables of the nf-fluid model (Sec. II-A states the two-fluid system
   with a continuity and a volume-fraction equation per component; this is
   the same system for nf components), stored in this order:
     0 .. nf-1          partial densities alpha_i rho_i
     nf, nf+1, nf+2     momentum rho u, rho v, rho w
     nf+3               total energy rho E
     nf+4 .. 2 nf+2     volume fractions alpha_1 .. alpha_{nf-1}
   with alpha_nf = 1 - (alpha_1 + ... + alpha_{nf-1}).  Two fluids give the
   seven variables (alpha1 rho1, alpha2 rho2, rho u, rho v, rho w, rho E,
   alpha1).  Primitives: the same with (u, v, w, p) in place of momentum
   and energy. */
static int nfl(const orc_grid* g) { return g->nf >= 2 ? g->nf : 2; }
static int nvar(const orc_grid* g) { return 2 * nfl(g) + 3; }
static int imom(const orc_grid* g) { return nfl(g); }
static int iene(const orc_grid* g) { return nfl(g) + 3; }
static int ialf(const orc_grid* g) { return nfl(g) + 4; }

/* ---------- equation of state (Sec. II-A) ---------- */

static double fluid_Gamma(const orc_grid* g, int f) { return 1.0 / (g->gamma[f] - 1.0); }
static double fluid_Pi(const orc_grid* g, int f)
{
    return g->gamma[f] * g->pinf[f] / (g->gamma[f] - 1.0);
}
/* Mixture rules, linear in the volume fractions a[0 .. nf-2] (the last
   fluid takes 1 minus their sum): sum_i alpha_i c_i of the per-fluid
   constants c_i.  For two fluids a1 c_1 + (1 - a1) c_2. */
static double mix_linear(const orc_grid* g, const double* a, int pi)
{
    const int nf = nfl(g);
    double m = 0.0, s = 0.0;
    for (int i = 0; i < nf - 1; ++i) {
        m = m + a[i] * (pi ? fluid_Pi(g, i) : fluid_Gamma(g, i));
        s = s + a[i];
    }
    return m + (1.0 - s) * (pi ? fluid_Pi(g, nf - 1) : fluid_Gamma(g, nf - 1));
}
/* mixture 1/(gamma-1) */
static double mix_Gamma(const orc_grid* g, const double* a) { return mix_linear(g, a, 0); }
/* mixture gamma*pi_inf/(gamma-1) */
static double mix_Pi(const orc_grid* g, const double* a) { return mix_linear(g, a, 1); }

static double mix_density(const orc_grid* g, const double* x)
{
    double rho = x[0];
    for (int i = 1; i < nfl(g); ++i) rho = rho + x[i];
    return rho;
}

static void cons_to_prim(const orc_grid* g, const double* q, double* w)
{
    const int m = imom(g), e = iene(g), a = ialf(g);
    double rho = mix_density(g, q);
    double ir = 1.0 / rho;
    double u = q[m] * ir, v = q[m + 1] * ir, ww = q[m + 2] * ir;
    double ke = 0.5 * rho * (u * u + v * v + ww * ww);
    double G = mix_Gamma(g, q + a), P = mix_Pi(g, q + a);
    for (int i = 0; i < nvar(g); ++i) w[i] = q[i];
    w[m] = u;
    w[m + 1] = v;
    w[m + 2] = ww;
    w[e] = (q[e] - ke - P) / G;
}

static void prim_to_cons(const orc_grid* g, const double* w, double* q)
{
    const int m = imom(g), e = iene(g), a = ialf(g);
    double rho = mix_density(g, w);
    double ke = 0.5 * rho * (w[m] * w[m] + w[m + 1] * w[m + 1] + w[m + 2] * w[m + 2]);
    for (int i = 0; i < nvar(g); ++i) q[i] = w[i];
    q[m] = rho * w[m];
    q[m + 1] = rho * w[m + 1];
    q[m + 2] = rho * w[m + 2];
    q[e] = mix_Gamma(g, w + a) * w[e] + mix_Pi(g, w + a) + ke;
}

/* c^2 = ((Gamma+1) p + Pi) / (Gamma rho); for one pure fluid this is
   gamma (p + pi_inf) / rho. */
static double sound_speed(const orc_grid* g, const double* w)
{
    double rho = mix_density(g, w);
    double G = mix_Gamma(g, w + ialf(g)), P = mix_Pi(g, w + ialf(g));
    return sqrt(((G + 1.0) * w[iene(g)] + P) / (G * rho));
}

/* ---------- WENO5 (Jiang-Shu weights) ----------
   Cell c with stencil values v[0..4] = w_{c-2..c+2}.  The three
   smoothness indicators belong to the cell and serve both of its edges.
   right = value at c+1/2 (linear weights 1/10, 6/10, 3/10 on the stencils
   {c-2..c}, {c-1..c+1}, {c..c+2}); left = value at c-1/2 (weights 3/10,
   6/10, 1/10 on the same stencils).  The indicators are those of Jiang &
   Shu: for each stencil, h times the cell integral of the squared first
   derivative plus h^3 times that of the squared second derivative of the
   stencil's quadratic. */
static void weno5_betas(const double* v, double* b)
{
    b[0] = 13.0 / 12.0 * (v[0] - 2.0 * v[1] + v[2]) * (v[0] - 2.0 * v[1] + v[2]) +
           0.25 * (v[0] - 4.0 * v[1] + 3.0 * v[2]) * (v[0] - 4.0 * v[1] + 3.0 * v[2]);
    b[1] = 13.0 / 12.0 * (v[1] - 2.0 * v[2] + v[3]) * (v[1] - 2.0 * v[2] + v[3]) +
           0.25 * (v[1] - v[3]) * (v[1] - v[3]);
    b[2] = 13.0 / 12.0 * (v[2] - 2.0 * v[3] + v[4]) * (v[2] - 2.0 * v[3] + v[4]) +
           0.25 * (3.0 * v[2] - 4.0 * v[3] + v[4]) * (3.0 * v[2] - 4.0 * v[3] + v[4]);
}

/* WENO-Z weights (Borges, Carmona, Costa & Don, J. Comput. Phys. 227, 2008),
   exponent 1: alpha_k = d_k (1 + tau5 / (beta_k + eps)), tau5 = |beta0 - beta2|.
   A comparison form, not the paper's method; same candidates and stencils. */
static void weno5_z(const double* v, double eps, double* left, double* right)
{
    double b[3];
    weno5_betas(v, b);
    double tau = fabs(b[0] - b[2]);

    double r0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    double r1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    double r2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
    double a0 = 0.1 * (1.0 + tau / (b[0] + eps));
    double a1 = 0.6 * (1.0 + tau / (b[1] + eps));
    double a2 = 0.3 * (1.0 + tau / (b[2] + eps));
    double s = a0 + a1 + a2;
    *right = (a0 / s) * r0 + (a1 / s) * r1 + (a2 / s) * r2;

    double l0 = (-v[0] + 5.0 * v[1] + 2.0 * v[2]) / 6.0;
    double l1 = (2.0 * v[1] + 5.0 * v[2] - v[3]) / 6.0;
    double l2 = (11.0 * v[2] - 7.0 * v[3] + 2.0 * v[4]) / 6.0;
    a0 = 0.3 * (1.0 + tau / (b[0] + eps));
    a1 = 0.6 * (1.0 + tau / (b[1] + eps));
    a2 = 0.1 * (1.0 + tau / (b[2] + eps));
    s = a0 + a1 + a2;
    *left = (a0 / s) * l0 + (a1 / s) * l1 + (a2 / s) * l2;
}

static void weno5(const double* v, double eps, double* left, double* right)
{
    double b[3];
    weno5_betas(v, b);
    double b0 = b[0], b1 = b[1], b2 = b[2];

    /* right edge c+1/2 */
    double r0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    double r1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    double r2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
    double a0 = 0.1 / ((eps + b0) * (eps + b0));
    double a1 = 0.6 / ((eps + b1) * (eps + b1));
    double a2 = 0.3 / ((eps + b2) * (eps + b2));
    double s = a0 + a1 + a2;
    *right = (a0 / s) * r0 + (a1 / s) * r1 + (a2 / s) * r2;

    /* left edge c-1/2 */
    double l0 = (-v[0] + 5.0 * v[1] + 2.0 * v[2]) / 6.0;
    double l1 = (2.0 * v[1] + 5.0 * v[2] - v[3]) / 6.0;
    double l2 = (11.0 * v[2] - 7.0 * v[3] + 2.0 * v[4]) / 6.0;
    a0 = 0.3 / ((eps + b0) * (eps + b0));
    a1 = 0.6 / ((eps + b1) * (eps + b1));
    a2 = 0.1 / ((eps + b2) * (eps + b2));
    s = a0 + a1 + a2;
    *left = (a0 / s) * l0 + (a1 / s) * l1 + (a2 / s) * l2;
}

/* WENO3 with Jiang-Shu weights (the third-order reconstruction Sec. II-B
   names beside WENO5; Jiang & Shu 1996, Shu 2006).  Cell c with stencil
   values v[0..2] = w_{c-1..c+1}; two candidate stencils {c-1, c} and
   {c, c+1}.  right = value at c+1/2 (candidates -v0/2 + 3v1/2 and
   v1/2 + v2/2, linear weights 1/3, 2/3); left = value at c-1/2 (candidates
   v0/2 + v1/2 and 3v1/2 - v2/2, linear weights 2/3, 1/3).  Indicators:
   the squared undivided differences of the two stencils. */
static void weno3(const double* v, double eps, double* left, double* right)
{
    double b0 = (v[1] - v[0]) * (v[1] - v[0]);
    double b1 = (v[2] - v[1]) * (v[2] - v[1]);

    double r0 = -0.5 * v[0] + 1.5 * v[1];
    double r1 = 0.5 * v[1] + 0.5 * v[2];
    double a0 = (1.0 / 3.0) / ((eps + b0) * (eps + b0));
    double a1 = (2.0 / 3.0) / ((eps + b1) * (eps + b1));
    double s = a0 + a1;
    *right = (a0 / s) * r0 + (a1 / s) * r1;

    double l0 = 0.5 * v[0] + 0.5 * v[1];
    double l1 = 1.5 * v[1] - 0.5 * v[2];
    a0 = (2.0 / 3.0) / ((eps + b0) * (eps + b0));
    a1 = (1.0 / 3.0) / ((eps + b1) * (eps + b1));
    s = a0 + a1;
    *left = (a0 / s) * l0 + (a1 / s) * l1;
}

/* Face states of the middle cell of a 5-value stencil in the grid's
   reconstruction: WENO5 (Jiang-Shu or WENO-Z weights), or WENO3 on the
   middle three values. */
/* ---------- WENO5 on non-uniform cells (Jiang-Shu weights) ----------
   The paper's mesh is structured with local refinement by a hyperbolic
   tangent stretching (Sec. III-A, Vinokur); the same reconstruction on cells
   of unequal widths, from its definition: cell c with stencil values
   v[0..4] (cell averages of cells c-2..c+2) and widths h[0..4].  In the
   coordinate xi = (x - x_c) / h_c (cell c spans [-1/2, 1/2]):
     candidate k (cells c-2+k .. c+k): the quadratic A + B xi + C xi^2 whose
       averages over those three cells are their values; its values at
       xi = 1/2 (right edge) and -1/2 (left edge);
     indicator beta_k = h_c int_c (p')^2 dx + h_c^3 int_c (p'')^2 dx
       = B^2 + 13/3 C^2;
     ideal weights d_k of an edge: the combination of the three candidates
       that equals the quartic through all five averages at that edge (the
       outer coefficients fix d_0 and d_2, the middle one d_1);
     alpha_k = d_k / (eps + beta_k)^2, omega = alpha / sum alpha.
   On equal widths this is weno5(). */

/* Solve the m x m system K y = r (m <= 5) by Gaussian elimination with
   partial pivoting; K and r are overwritten. */
static void solve_small(int m, double K[5][5], double* r)
{
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int i = c + 1; i < m; ++i)
            if (fabs(K[i][c]) > fabs(K[p][c])) p = i;
        for (int j = 0; j < m; ++j) {
            const double t = K[c][j];
            K[c][j] = K[p][j];
            K[p][j] = t;
        }
        const double t = r[c];
        r[c] = r[p];
        r[p] = t;
        for (int i = c + 1; i < m; ++i) {
            const double f = K[i][c] / K[c][c];
            for (int j = c; j < m; ++j) K[i][j] = K[i][j] - f * K[c][j];
            r[i] = r[i] - f * r[c];
        }
    }
    for (int c = m - 1; c >= 0; --c) {
        double a = r[c];
        for (int j = c + 1; j < m; ++j) a = a - K[c][j] * r[j];
        r[c] = a / K[c][c];
    }
}

/* Cell boundaries of cells c-2..c+2 in the coordinate xi of cell c. */
static void stencil_bounds(const double* h, double lo[5], double hi[5])
{
    lo[2] = -0.5;
    hi[2] = 0.5;
    for (int k = 1; k >= 0; --k) {
        hi[k] = lo[k + 1];
        lo[k] = hi[k] - h[k] / h[2];
    }
    for (int k = 3; k < 5; ++k) {
        lo[k] = hi[k - 1];
        hi[k] = lo[k] + h[k] / h[2];
    }
}

/* Average of xi^m over [a, b]. */
static double avg_pow(int m, double a, double b)
{
    return (pow(b, m + 1) - pow(a, m + 1)) / ((m + 1) * (b - a));
}

/* Coefficients g[j] of the value at xi = x0 of the polynomial of degree
   m-1 whose averages over cells first .. first+m-1 are the values v: the
   value is sum_j g[j] v[first+j]. */
static void face_row(int m, int first, const double lo[5], const double hi[5], double x0, double* gout)
{
    double K[5][5], r[5];
    /* K^T g = phi, with K[i][e] = average of xi^e over cell first+i */
    for (int e = 0; e < m; ++e) {
        for (int i = 0; i < m; ++i) K[e][i] = avg_pow(e, lo[first + i], hi[first + i]);
        r[e] = pow(x0, e);
    }
    solve_small(m, K, r);
    for (int i = 0; i < m; ++i) gout[i] = r[i];
}

/* Ideal weights of the edge at xi = x0. */
static void ideal_weights(const double lo[5], const double hi[5], double x0, double d[3])
{
    double g5[5], r0[3], r1[3], r2[3];
    face_row(5, 0, lo, hi, x0, g5);
    face_row(3, 0, lo, hi, x0, r0);
    face_row(3, 1, lo, hi, x0, r1);
    face_row(3, 2, lo, hi, x0, r2);
    d[0] = g5[0] / r0[0];
    d[2] = g5[4] / r2[2];
    d[1] = (g5[2] - d[0] * r0[2] - d[2] * r2[0]) / r1[1];
}

static void weno5_nu(const double* h, const double* v, double eps, double* left, double* right)
{
    double lo[5], hi[5];
    stencil_bounds(h, lo, hi);
    double beta[3], pr[3], pl[3];
    for (int k = 0; k < 3; ++k) {
        double K[5][5], y[5];
        for (int i = 0; i < 3; ++i) {
            for (int e = 0; e < 3; ++e) K[i][e] = avg_pow(e, lo[k + i], hi[k + i]);
            y[i] = v[k + i];
        }
        solve_small(3, K, y); /* y = (A, B, C) */
        beta[k] = y[1] * y[1] + 13.0 / 3.0 * (y[2] * y[2]);
        pr[k] = y[0] + 0.5 * y[1] + 0.25 * y[2];
        pl[k] = y[0] - 0.5 * y[1] + 0.25 * y[2];
    }
    double dr[3], dl[3];
    ideal_weights(lo, hi, 0.5, dr);
    ideal_weights(lo, hi, -0.5, dl);
    double ar[3], al[3], sr = 0.0, sl = 0.0;
    for (int k = 0; k < 3; ++k) {
        ar[k] = dr[k] / ((eps + beta[k]) * (eps + beta[k]));
        al[k] = dl[k] / ((eps + beta[k]) * (eps + beta[k]));
        sr += ar[k];
        sl += al[k];
    }
    *right = (ar[0] / sr) * pr[0] + (ar[1] / sr) * pr[1] + (ar[2] / sr) * pr[2];
    *left = (al[0] / sl) * pl[0] + (al[1] / sl) * pl[1] + (al[2] / sl) * pl[2];
}

static void reconstruct(const orc_grid* g, const double* st, double* left, double* right)
{
    if (g->weno_order == 3)
        weno3(st + 1, g->eps, left, right);
    else if (g->weno_z)
        weno5_z(st, g->eps, left, right);
    else
        weno5(st, g->eps, left, right);
}

/* ---------- HLLC (Toro 2009, Davis wave speeds) ----------
   Face with normal along direction d; wl, wr primitive states.  Returns
   the flux of every variable and the face velocity used for div(u).  In
   the star state every partial density and every volume fraction is
   scaled by xi. */
static void hllc(const orc_grid* g, const double* wl, const double* wr, int d, double* F,
                 double* uf)
{
    const int nv = nvar(g), m = imom(g), e = iene(g), a = ialf(g), nf = nfl(g);
    double rl = mix_density(g, wl), rr = mix_density(g, wr);
    double pl = wl[e], pr = wr[e];
    double unl = wl[m + d], unr = wr[m + d];
    double El = mix_Gamma(g, wl + a) * pl + mix_Pi(g, wl + a) +
                0.5 * rl * (wl[m] * wl[m] + wl[m + 1] * wl[m + 1] + wl[m + 2] * wl[m + 2]);
    double Er = mix_Gamma(g, wr + a) * pr + mix_Pi(g, wr + a) +
                0.5 * rr * (wr[m] * wr[m] + wr[m + 1] * wr[m + 1] + wr[m + 2] * wr[m + 2]);
    double cl = sound_speed(g, wl), cr = sound_speed(g, wr);

    double SL = fmin(unl - cl, unr - cr);
    double SR = fmax(unl + cl, unr + cr);
    double Ss = (pr - pl + rl * unl * (SL - unl) - rr * unr * (SR - unr)) /
                (rl * (SL - unl) - rr * (SR - unr));

    /* pick the side of the contact (ties go left) */
    const double* w;
    double rho, p, un, E, S, s;
    if (Ss >= 0.0) {
        w = wl; rho = rl; p = pl; un = unl; E = El; S = SL; s = fmin(0.0, SL);
    } else {
        w = wr; rho = rr; p = pr; un = unr; E = Er; S = SR; s = fmax(0.0, SR);
    }

    double U[NVMAX], Fk[NVMAX], Us[NVMAX];
    for (int i = 0; i < nf; ++i) U[i] = w[i];
    U[m] = rho * w[m];
    U[m + 1] = rho * w[m + 1];
    U[m + 2] = rho * w[m + 2];
    U[e] = E;
    for (int i = a; i < nv; ++i) U[i] = w[i];

    for (int v = 0; v < nv; ++v) Fk[v] = U[v] * un;
    Fk[m + d] = Fk[m + d] + p;
    Fk[e] = (E + p) * un;

    /* xi = (S - u)/(S - S*); the star energy's pressure term
       xi (S* - u) p/(S - u) is (S* - u) p/(S - S*), so one quotient serves both */
    double inv = 1.0 / (S - Ss);
    double xi = (S - un) * inv;
    for (int i = 0; i < nf; ++i) Us[i] = xi * w[i];
    Us[m] = xi * (rho * w[m]);
    Us[m + 1] = xi * (rho * w[m + 1]);
    Us[m + 2] = xi * (rho * w[m + 2]);
    Us[m + d] = xi * (rho * Ss);
    Us[e] = xi * (E + (Ss - un) * (rho * Ss)) + (Ss - un) * (p * inv);
    for (int i = a; i < nv; ++i) Us[i] = xi * w[i];

    for (int v = 0; v < nv; ++v) F[v] = Fk[v] + s * (Us[v] - U[v]);
    *uf = un + s * (xi - 1.0);
}

/* ---------- boundary index map ----------
   The cell whose state ghost cell i (outside 0..n-1) takes: periodic wraps
   around, transmissive repeats the edge cell (zero gradient), reflective
   mirrors about the boundary face (ghost -1-k <- cell k, ghost n+k <- cell
   n-1-k) and sets *flip: that ghost carries the mirrored cell's state with
   the momentum normal to the wall negated (a stationary slip wall; the
   paper names no boundary type, this is the standard ghost construction).
   Reflective sides need n >= 3 (checked by the Python wrapper).  An inflow
   side sets *flip = 2: its ghosts hold the side's fixed state
   (g->inflow[d][side]) instead of a cell's (the returned index is the
   edge cell, a placeholder). */
static int64_t map_index(const orc_grid* g, int d, int64_t i, int* flip)
{
    int64_t n = g->n[d];
    *flip = 0;
    if (i >= 0 && i < n) return i;
    int t = g->bc[d][i < 0 ? 0 : 1];
    if (t == 2) {
        *flip = 1;
        return i < 0 ? -1 - i : 2 * n - 1 - i;
    }
    if (t == 3) *flip = 2;
    if (i < 0) return t == 0 ? ((i % n) + n) % n : 0;
    return t == 0 ? i % n : n - 1;
}

/* Ghost state adjustment for what map_index reported: reflective ghosts
   negate the momentum normal to the wall, inflow ghosts take the side's
   fixed state. */
static void ghost_state(const orc_grid* g, int d, int64_t i, int kind, double* qc)
{
    if (kind == 1) qc[imom(g) + d] = -qc[imom(g) + d];
    if (kind == 2)
        for (int v = 0; v < nvar(g); ++v) qc[v] = g->inflow[d][i < 0 ? 0 : 1][v];
}

static int active(const orc_grid* g, int d) { return g->n[d] > 1; }

/* Width of cell i along d; a ghost cell takes the width of the cell whose
   state the boundary map gives it (periodic: the wrapped cell; transmissive
   and inflow: the edge cell; reflective: the mirrored cell). */
static double cell_width(const orc_grid* g, int d, int64_t i)
{
    if (!g->xf[d]) return g->dx[d];
    int flip;
    const int64_t j = map_index(g, d, i, &flip);
    return g->xf[d][j + 1] - g->xf[d][j];
}

/* Face states of the middle cell of a stencil at position c along d:
   WENO5 on the cells' widths for a non-uniform direction, else the grid's
   uniform reconstruction. */
static void reconstruct_at(const orc_grid* g, int d, int64_t c, const double* st, double* left, double* right)
{
    if (g->xf[d]) {
        double h[5];
        for (int o = 0; o < 5; ++o) h[o] = cell_width(g, d, c - 2 + o);
        weno5_nu(h, st, g->eps, left, right);
    } else {
        reconstruct(g, st, left, right);
    }
}

/* ---------- exported helpers for unit tests ---------- */
void orc_weno5(const double* v, double eps, double* left, double* right)
{
    weno5(v, eps, left, right);
}
void orc_weno5_betas(const double* v, double* b) { weno5_betas(v, b); }
void orc_weno5_z(const double* v, double eps, double* left, double* right) { weno5_z(v, eps, left, right); }
void orc_weno3(const double* v, double eps, double* left, double* right) { weno3(v, eps, left, right); }
void orc_weno5_nu(const double* h, const double* v, double eps, double* left, double* right)
{
    weno5_nu(h, v, eps, left, right);
}
/* Indicators beta_k of the middle cell of five cells of widths h (pins). */
void orc_weno5_nu_betas(const double* h, const double* v, double* beta)
{
    double lo[5], hi[5];
    stencil_bounds(h, lo, hi);
    for (int k = 0; k < 3; ++k) {
        double K[5][5], y[5];
        for (int i = 0; i < 3; ++i) {
            for (int e = 0; e < 3; ++e) K[i][e] = avg_pow(e, lo[k + i], hi[k + i]);
            y[i] = v[k + i];
        }
        solve_small(3, K, y);
        beta[k] = y[1] * y[1] + 13.0 / 3.0 * (y[2] * y[2]);
    }
}

/* Ideal weights of the right and left edge of the middle cell of five cells
   of widths h (pins). */
void orc_ideal_weights_nu(const double* h, double* dr, double* dl)
{
    double lo[5], hi[5];
    stencil_bounds(h, lo, hi);
    ideal_weights(lo, hi, 0.5, dr);
    ideal_weights(lo, hi, -0.5, dl);
}
void orc_hllc(const orc_grid* g, const double* wl, const double* wr, int d, double* F, double* uf)
{
    hllc(g, wl, wr, d, F, uf);
}
double orc_sound_speed(const orc_grid* g, const double* w) { return sound_speed(g, w); }
void orc_cons_to_prim_cell(const orc_grid* g, const double* q, double* w) { cons_to_prim(g, q, w); }
void orc_prim_to_cons_cell(const orc_grid* g, const double* w, double* q) { prim_to_cons(g, w, q); }

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads a parallel region of the oracle actually runs with. */
int orc_team_size(void)
{
    int n = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
#endif
    return n;
}

/* Thread count of later parallel regions (timing only; results do not
   depend on it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int64_t ncells(const orc_grid* g) { return (int64_t)g->n[0] * g->n[1] * g->n[2]; }

/* Whole-array conversions, layout [nvar][nz][ny][nx]. */
void orc_prim_to_cons(const orc_grid* g, const double* w, double* q)
{
    int64_t N = ncells(g);
    const int nv = nvar(g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        double wc[NVMAX], qc[NVMAX];
        for (int v = 0; v < nv; ++v) wc[v] = w[v * N + c];
        prim_to_cons(g, wc, qc);
        for (int v = 0; v < nv; ++v) q[v * N + c] = qc[v];
    }
}

void orc_cons_to_prim(const orc_grid* g, const double* q, double* w)
{
    int64_t N = ncells(g);
    const int nv = nvar(g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        double wc[NVMAX], qc[NVMAX];
        for (int v = 0; v < nv; ++v) qc[v] = q[v * N + c];
        cons_to_prim(g, qc, wc);
        for (int v = 0; v < nv; ++v) w[v * N + c] = wc[v];
    }
}

/* ---------- learned WENO weights (an addition to the paper's method) ----------
   The paper's WENO5 (Sec. II-B) with the Jiang-Shu weights corrected by a
   small network, as the solver applies it:
     features of a 5-value stencil v reconstructed at its right edge, with
     the Jiang-Shu indicators beta_k and S = beta0 + beta1 + beta2 + eps:
       x = (beta0/S, beta1/S, beta2/S, |beta0 - beta2|/S, D^2/(S + D^2)),
       D = v0 - 4 v1 + 6 v2 - 4 v3 + v4;
     network 5 -> 32 -> 32 -> 3 with GELU (trained with its tanh form
       a (1 + tanh(sqrt(2/pi) (a + 0.044715 a^3))) / 2), evaluated at
       inference as max(a, 0) - t Q(t), t = min(|a|, 3.75), Q a degree-6
       polynomial fitted (minimax) to the tanh form's remainder
       h(t) = t (1 - tanh(sqrt(2/pi) (t + 0.044715 t^3))) / 2, within
       1.2e-4 of the tanh form (see gelu_inference), giving logits z; weights omega = softmax(ln omega_JS + z) on the three
     third-order candidates (a zero output layer is Jiang-Shu);
     a cell's left edge is the right edge of its reversed stencil.
   Inference precision of the method: the features, the weights of all
   three layers, the first layer's bias and both hidden activations are
   rounded to bfloat16 (through float32, nearest, ties to even); the second
   and third layers' biases stay as given (float32 values); sums, softmax
   and candidates are evaluated here in float64.
   Two forms:
     per variable (mode 1): every variable and edge evaluates the network on
       its own stencil;
     shared per edge (mode 2): one evaluation per edge for all seven
       variables, on the componentwise maximum of their features; its logits
       correct each variable's own Jiang-Shu weights, so a zero output
       layer is Jiang-Shu for every variable.
   Fallback per edge: if any weight of the edge is not finite, or its
   learned state (all seven primitives) is not admissible -- a negative
   partial density, alpha1 outside [0, 1], (Gamma + 1) p + Pi <= 0, or a
   non-finite value -- every variable of that edge takes its Jiang-Shu
   value. */
#define MLP_H 32

typedef struct {
    double W1[MLP_H][5], b1[MLP_H], W2[MLP_H][MLP_H], b2[MLP_H], W3[3][MLP_H], b3[3];
} orc_mlp;

/* float64 -> float32 -> bfloat16 (round to nearest, ties to even), back as double */
static double bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double gelu_tanh(double a)
{
    const double c = sqrt(2.0 / 3.14159265358979323846); /* sqrt(2 / pi) */
    return 0.5 * a * (1.0 + tanh(c * (a + 0.044715 * a * a * a)));
}

/* GELU as the inference evaluates it: the positive part of a minus the
   tanh form's remainder h(|a|), h replaced beyond 3.75 by its value there
   and below by t Q(t) with Q(t) = q0 + q1 t + ... + q6 t^6 (coefficients as
   float32 values, the definition of the inference network). */
static double gelu_inference(double a)
{
    static const double q[7] = {0.497150153, -0.375513077, -0.0665387958, 0.157749414,
                                -0.0645674914, 0.0113088572, -0.00075154379};
    const double t = fmin(fabs(a), 3.75);
    double Q = 0.0, tk = 1.0;
    for (int k = 0; k < 7; ++k) {
        Q += (double)(float)q[k] * tk;
        tk *= t;
    }
    return fmax(a, 0.0) - t * Q;
}

/* Parameters in the order W1[32][5], b1[32], W2[32][32], b2[32], W3[3][32],
   b3[3], with the bfloat16 rounding of the operands applied once. */
static void mlp_load(const double* theta, orc_mlp* m)
{
    int o = 0;
    for (int j = 0; j < MLP_H; ++j)
        for (int k = 0; k < 5; ++k) m->W1[j][k] = bf16(theta[o++]);
    for (int j = 0; j < MLP_H; ++j) m->b1[j] = bf16(theta[o++]);
    for (int j = 0; j < MLP_H; ++j)
        for (int k = 0; k < MLP_H; ++k) m->W2[j][k] = bf16(theta[o++]);
    for (int j = 0; j < MLP_H; ++j) m->b2[j] = theta[o++];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < MLP_H; ++k) m->W3[i][k] = bf16(theta[o++]);
    for (int i = 0; i < 3; ++i) m->b3[i] = theta[o++];
}

/* Logits of one feature vector (operands in bfloat16 as above). */
static void mlp_logits(const orc_mlp* m, const double x[5], double z[3])
{
    double xb[5], h1[MLP_H], h2[MLP_H];
    for (int k = 0; k < 5; ++k) xb[k] = bf16(x[k]);
    for (int j = 0; j < MLP_H; ++j) {
        double a = m->b1[j];
        for (int k = 0; k < 5; ++k) a += m->W1[j][k] * xb[k];
        h1[j] = bf16(gelu_inference(a));
    }
    for (int j = 0; j < MLP_H; ++j) {
        double a = m->b2[j];
        for (int k = 0; k < MLP_H; ++k) a += m->W2[j][k] * h1[k];
        h2[j] = bf16(gelu_inference(a));
    }
    for (int i = 0; i < 3; ++i) {
        double a = m->b3[i];
        for (int k = 0; k < MLP_H; ++k) a += m->W3[i][k] * h2[k];
        z[i] = a;
    }
}

/* Right-edge statistics of a stencil: features, normalised Jiang-Shu
   weights, candidate values. */
static void right_edge_stats(const double* v, double eps, double x[5], double ojs[3], double cand[3])
{
    double b[3];
    weno5_betas(v, b);
    const double S = b[0] + b[1] + b[2] + eps;
    const double D = v[0] - 4.0 * v[1] + 6.0 * v[2] - 4.0 * v[3] + v[4];
    x[0] = b[0] / S;
    x[1] = b[1] / S;
    x[2] = b[2] / S;
    x[3] = fabs(b[0] - b[2]) / S;
    x[4] = D * D / (S + D * D);
    const double a0 = 0.1 / ((eps + b[0]) * (eps + b[0]));
    const double a1 = 0.6 / ((eps + b[1]) * (eps + b[1]));
    const double a2 = 0.3 / ((eps + b[2]) * (eps + b[2]));
    const double s = a0 + a1 + a2;
    ojs[0] = a0 / s;
    ojs[1] = a1 / s;
    ojs[2] = a2 / s;
    cand[0] = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    cand[1] = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    cand[2] = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
}

/* omega = softmax(ln base + z); returns 0 if a weight is not finite */
static int corrected_weights(const double base[3], const double z[3], double om[3])
{
    double l[3], lm = -INFINITY;
    for (int k = 0; k < 3; ++k) {
        l[k] = log(base[k]) + z[k];
        if (l[k] > lm) lm = l[k];
    }
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        om[k] = exp(l[k] - lm);
        s += om[k];
    }
    int fin = 1;
    for (int k = 0; k < 3; ++k) {
        om[k] = om[k] / s;
        fin = fin && isfinite(om[k]);
    }
    return fin;
}

/* Admissibility of an edge state w (primitives).  *near is set when a test
   is decided by a margin another evaluation could cross: 2^-20 of the
   stencil's magnitude (scale[v], the largest |value| of variable v's
   stencil; float32 rounding) plus 1/32 of the spread of its candidates
   (spread[v]; a few per cent change of the weights, as a bfloat16 rounding
   of an operand of the network can cause). */
static int admissible_edge(const orc_grid* g, const double w[NV], const double scale[NV], const double spread[NV],
                           int* near)
{
    const double G = mix_Gamma(g, w + 6), P = mix_Pi(g, w + 6);
    const double c2n = (G + 1.0) * w[5] + P;
    int fin = 1;
    for (int v = 0; v < NV; ++v) fin = fin && isfinite(w[v]);
    const int ok = fin && w[0] >= 0.0 && w[1] >= 0.0 && w[6] >= 0.0 && w[6] <= 1.0 && c2n > 0.0;
    double m[NV];
    for (int v = 0; v < NV; ++v) m[v] = 0x1p-20 * scale[v] + 0x1p-5 * spread[v];
    const double dG = fabs(fluid_Gamma(g, 0) - fluid_Gamma(g, 1)), dP = fabs(fluid_Pi(g, 0) - fluid_Pi(g, 1));
    const double mc = 0x1p-20 * (fabs((G + 1.0) * w[5]) + fabs(P)) +
                      fabs(G + 1.0) * m[5] + (dG * fabs(w[5]) + dP) * m[6];
    if (fin && (fabs(w[0]) <= m[0] || fabs(w[1]) <= m[1] || fabs(w[6]) <= m[6] || fabs(w[6] - 1.0) <= m[6] ||
                fabs(c2n) <= mc))
        *near = 1;
    return ok;
}

typedef struct {
    const orc_mlp* m;
    int mode;       /* 1 per variable, 2 shared per edge */
    int plant;      /* tests only: a deliberate mistake (0 none), see orc_rhs_learned */
} orc_learn;

/* Both edge states of one cell (all seven variables) from its stencils
   st[v][0..4] with learned weights.  fb[0], fb[1]: the right and left edge
   fell back; nr[0], nr[1]: the decision was near a threshold. */
static void learned_cell(const orc_grid* g, const orc_learn* L, double st[NV][5], double* lft, double* rgt, int fb[2],
                         int nr[2])
{
    double scale[NV];
    double jl[NV], jr[NV];
    for (int v = 0; v < NV; ++v) {
        weno5(st[v], g->eps, &jl[v], &jr[v]);
        scale[v] = 0.0;
        for (int k = 0; k < 5; ++k)
            if (fabs(st[v][k]) > scale[v]) scale[v] = fabs(st[v][k]);
    }
    /* side 0: right edge (the stencil as it is); side 1: left edge (the
       reversed stencil's right edge) */
    double val[2][NV];
    int fin[2] = {1, 1};
    double X[2][NV][5], O[2][NV][3], C[2][NV][3];
    for (int side = 0; side < 2; ++side)
        for (int v = 0; v < NV; ++v) {
            double sv[5];
            for (int k = 0; k < 5; ++k) sv[k] = side == 0 ? st[v][k] : st[v][4 - k];
            right_edge_stats(sv, g->eps, X[side][v], O[side][v], C[side][v]);
        }
    if (L->plant == 1) /* mistake: the left edge takes the unreversed stencil's features */
        for (int v = 0; v < NV; ++v)
            for (int k = 0; k < 5; ++k) X[1][v][k] = X[0][v][k];
    for (int side = 0; side < 2; ++side) {
        if (L->mode == 2) {
            double f[5], z[3];
            for (int k = 0; k < 5; ++k) {
                f[k] = X[side][0][k];
                for (int v = 1; v < NV; ++v)
                    if (X[side][v][k] > f[k]) f[k] = X[side][v][k];
            }
            mlp_logits(L->m, f, z);
            double pooled[3], ps = 0.0;
            if (L->plant == 4) { /* mistake: one baseline for all variables, their weights' minimum */
                for (int k = 0; k < 3; ++k) {
                    pooled[k] = O[side][0][k];
                    for (int v = 1; v < NV; ++v)
                        if (O[side][v][k] < pooled[k]) pooled[k] = O[side][v][k];
                    ps += pooled[k];
                }
                for (int k = 0; k < 3; ++k) pooled[k] /= ps;
            }
            for (int v = 0; v < NV; ++v) {
                double om[3];
                fin[side] = corrected_weights(L->plant == 4 ? pooled : O[side][v], z, om) && fin[side];
                val[side][v] = om[0] * C[side][v][0] + om[1] * C[side][v][1] + om[2] * C[side][v][2];
            }
        } else {
            for (int v = 0; v < NV; ++v) {
                double z[3], om[3];
                mlp_logits(L->m, X[side][v], z);
                fin[side] = corrected_weights(O[side][v], z, om) && fin[side];
                val[side][v] = om[0] * C[side][v][0] + om[1] * C[side][v][1] + om[2] * C[side][v][2];
            }
        }
    }
    for (int side = 0; side < 2; ++side) {
        double spread[NV];
        for (int v = 0; v < NV; ++v) {
            const double* c = C[side][v];
            spread[v] = fmax(c[0], fmax(c[1], c[2])) - fmin(c[0], fmin(c[1], c[2]));
        }
        nr[side] = 0;
        const int ok = fin[side] && admissible_edge(g, val[side], scale, spread, &nr[side]);
        fb[side] = !ok;
        double* out = side == 0 ? rgt : lft;
        const double* js = side == 0 ? jr : jl;
        if (L->plant == 3) { /* mistake: fallback per variable (only the variables that fail their own test) */
            const double* w = val[side];
            const double c2n = (mix_Gamma(g, w + 6) + 1.0) * w[5] + mix_Pi(g, w + 6);
            for (int v = 0; v < NV; ++v) {
                int vok = fin[side] && isfinite(w[v]);
                if (v == 0 || v == 1) vok = vok && w[v] >= 0.0;
                if (v == 6) vok = vok && w[6] >= 0.0 && w[6] <= 1.0;
                if (v == 5) vok = vok && c2n > 0.0;
                out[v] = vok ? w[v] : js[v];
            }
        } else {
            for (int v = 0; v < NV; ++v) out[v] = ok ? val[side][v] : js[v];
        }
    }
    if (L->plant == 2) /* mistake: the edges exchanged */
        for (int v = 0; v < NV; ++v) {
            const double t = lft[v];
            lft[v] = rgt[v];
            rgt[v] = t;
        }
}

/* ---------- right-hand side on the whole grid ----------
   L: learned weights (NULL for the grid's own reconstruction); counts[0]
   receives the edges that fell back (each edge a face uses, each distinct
   face once), counts[1] those whose decision was near a threshold. */
static void rhs_impl(const orc_grid* g, const double* q, double* rhs, const orc_learn* L, int64_t* counts)
{
    int gh[3], P[3];
    for (int d = 0; d < 3; ++d) {
        gh[d] = active(g, d) ? NG : 0;
        P[d] = g->n[d] + 2 * gh[d];
    }
    const int64_t N = ncells(g);
    const int64_t NP = (int64_t)P[0] * P[1] * P[2];
    const int nv = nvar(g), ia0 = ialf(g);
    double* wp = (double*)malloc(sizeof(double) * nv * NP);
    int64_t nfb = 0, nnear = 0;

    /* padded primitive array: ghosts filled by the BC map, then converted */
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < P[2]; ++k)
        for (int j = 0; j < P[1]; ++j) {
            int fk, fj, fi;
            int64_t sk = map_index(g, 2, k - gh[2], &fk);
            int64_t sj = map_index(g, 1, j - gh[1], &fj);
            for (int i = 0; i < P[0]; ++i) {
                int64_t si = map_index(g, 0, i - gh[0], &fi);
                int64_t src = (sk * g->n[1] + sj) * g->n[0] + si;
                int64_t dst = ((int64_t)k * P[1] + j) * P[0] + i;
                double qc[NVMAX], wc[NVMAX];
                for (int v = 0; v < nv; ++v) qc[v] = q[v * N + src];
                /* reflective and inflow ghosts, per direction */
                ghost_state(g, 0, i - gh[0], fi, qc);
                ghost_state(g, 1, j - gh[1], fj, qc);
                ghost_state(g, 2, k - gh[2], fk, qc);
                cons_to_prim(g, qc, wc);
                for (int v = 0; v < nv; ++v) wp[v * NP + dst] = wc[v];
            }
        }

    for (int64_t x = 0; x < nv * N; ++x) rhs[x] = 0.0;

    /* one sweep per active direction, in the order x, y, z */
    for (int d = 0; d < 3; ++d) {
        if (!active(g, d)) continue;
        int a = (d == 0) ? 1 : 0;          /* first transverse direction */
        int b = (d == 2) ? 1 : 2;          /* second transverse direction */
        int64_t stride_p[3] = {1, P[0], (int64_t)P[0] * P[1]};
        int64_t stride_n[3] = {1, g->n[0], (int64_t)g->n[0] * g->n[1]};
        int n = g->n[d];
        /* distinct faces of a pencil: with periodic ends faces 0 and n coincide */
        const int nfaces = g->bc[d][0] == 0 ? n : n + 1;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : nfb, nnear)
        for (int ib = 0; ib < g->n[b]; ++ib)
            for (int ia = 0; ia < g->n[a]; ++ia) {
                /* edges of cells -1..n, faces 0..n (face f sits between f-1 and f) */
                double* lft = (double*)malloc(sizeof(double) * nv * (n + 2));
                double* rgt = (double*)malloc(sizeof(double) * nv * (n + 2));
                double* F = (double*)malloc(sizeof(double) * nv * (n + 1));
                double* uf = (double*)malloc(sizeof(double) * (n + 1));
                int* flag = L ? (int*)malloc(sizeof(int) * 4 * (n + 2)) : NULL;
                int64_t base_p = (ia + gh[a]) * stride_p[a] + (ib + gh[b]) * stride_p[b];
                int64_t base_n = ia * stride_n[a] + ib * stride_n[b];
                for (int c = -1; c <= n; ++c) {
                    double st[NVMAX][5];
                    for (int v = 0; v < nv; ++v)
                        for (int o = -2; o <= 2; ++o)
                            st[v][o + 2] = wp[v * NP + base_p + (int64_t)(c + gh[d] + o) * stride_p[d]];
                    if (L) { /* two fluids (nv == NV) */
                        int* fl = &flag[4 * (c + 1)];
                        learned_cell(g, L, st, &lft[(c + 1) * nv], &rgt[(c + 1) * nv], fl, fl + 2);
                    } else {
                        for (int v = 0; v < nv; ++v)
                            reconstruct_at(g, d, c, st[v], &lft[(c + 1) * nv + v], &rgt[(c + 1) * nv + v]);
                    }
                }
                if (L) {
                    /* face f: right edge of cell f-1 (index f), left edge of cell f (index f+1) */
                    for (int f = 0; f < nfaces; ++f) {
                        nfb += flag[4 * f + 0] + flag[4 * (f + 1) + 1];
                        nnear += flag[4 * f + 2] + flag[4 * (f + 1) + 3];
                    }
                }
                for (int f = 0; f <= n; ++f)
                    hllc(g, &rgt[f * nv], &lft[(f + 1) * nv], d, &F[f * nv], &uf[f]);
                for (int i = 0; i < n; ++i) {
                    int64_t cell = base_n + (int64_t)i * stride_n[d];
                    const double h = cell_width(g, d, i);
                    for (int v = 0; v < nv; ++v)
                        rhs[v * N + cell] += (F[i * nv + v] - F[(i + 1) * nv + v]) / h;
                    /* every volume-fraction equation carries alpha_i div(u) */
                    for (int v = ia0; v < nv; ++v) {
                        double ai = wp[v * NP + base_p + (int64_t)(i + gh[d]) * stride_p[d]];
                        rhs[v * N + cell] += ai * ((uf[i + 1] - uf[i]) / h);
                    }
                }
                free(lft);
                free(rgt);
                free(F);
                free(uf);
                free(flag);
            }
    }
    free(wp);
    if (counts) {
        counts[0] = nfb;
        counts[1] = nnear;
    }
}

void orc_rhs(const orc_grid* g, const double* q, double* rhs) { rhs_impl(g, q, rhs, NULL, NULL); }

/* Right-hand side with learned WENO weights (fifth order; the grid's
   weno_z / weno_order are not used).  theta: the 1347 network parameters
   (float32 values); mode 1 per variable, 2 shared per edge; counts[2] as
   in rhs_impl (may be NULL).  plant (tests only, 0 otherwise) builds in a
   deliberate mistake to show what the comparisons catch: 1 the left edge
   takes the unreversed stencil's features, 2 the two edges exchanged, 3 the
   fallback per variable (only the variables that fail their own test take
   the Jiang-Shu value) instead of per edge, 4 the shared logits applied to
   one baseline for all variables (the renormalised componentwise minimum
   of their Jiang-Shu weights) instead of to each variable's own. */
void orc_rhs_learned(const orc_grid* g, const double* q, const double* theta, int mode, int plant, double* rhs,
                     int64_t* counts)
{
    if (nvar(g) != NV) { /* the learned weights are defined for two fluids */
        for (int64_t x = 0; x < nvar(g) * ncells(g); ++x) rhs[x] = NAN;
        return;
    }
    orc_mlp m;
    mlp_load(theta, &m);
    orc_learn L = {&m, mode == 2 ? 2 : 1, plant};
    rhs_impl(g, q, rhs, &L, counts);
}

/* Logits and weights of single samples (pins): features x[n][5], baseline
   base[n][3] -> omega[n][3] with the bfloat16 operands as in the solver. */
void orc_mlp_omega(const double* theta, int64_t n, const double* x, const double* base, double* omega)
{
    orc_mlp m;
    mlp_load(theta, &m);
    for (int64_t i = 0; i < n; ++i) {
        double z[3];
        mlp_logits(&m, x + 5 * i, z);
        corrected_weights(base + 3 * i, z, omega + 3 * i);
    }
}

double orc_gelu(double a) { return gelu_inference(a); }
double orc_gelu_tanh(double a) { return gelu_tanh(a); }

/* ---------- right-hand side at selected cells, one by one ----------
   cells: linear indices (k*ny + j)*nx + i; out: [ncell][nvar].  Uses the same
   per-cell formulas with the BC map applied to each stencil index, and the
   same accumulation order, so it equals orc_rhs at those cells (and, with
   learned weights L, orc_rhs_learned: the same learned_cell on the same
   stencils). */
static void rhs_at_impl(const orc_grid* g, const double* q, int64_t ncell, const int64_t* cells, double* out,
                        const orc_learn* L)
{
    const int64_t N = ncells(g);
    const int nv = nvar(g), ia0 = ialf(g);
    int64_t stride_n[3] = {1, g->n[0], (int64_t)g->n[0] * g->n[1]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < ncell; ++c) {
        int64_t lin = cells[c];
        int64_t pos[3] = {lin % g->n[0], (lin / g->n[0]) % g->n[1], lin / ((int64_t)g->n[0] * g->n[1])};
        double r[NVMAX];
        for (int v = 0; v < nv; ++v) r[v] = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (!active(g, d)) continue;
            double w7[7][NVMAX];
            for (int o = -3; o <= 3; ++o) {
                int64_t p2[3] = {pos[0], pos[1], pos[2]};
                int flip;
                p2[d] = map_index(g, d, pos[d] + o, &flip);
                int64_t src = p2[0] * stride_n[0] + p2[1] * stride_n[1] + p2[2] * stride_n[2];
                double qc[NVMAX];
                for (int v = 0; v < nv; ++v) qc[v] = q[v * N + src];
                ghost_state(g, d, pos[d] + o, flip, qc);
                cons_to_prim(g, qc, w7[o + 3]);
            }
            double lft[3][NVMAX], rgt[3][NVMAX];
            for (int cc = 0; cc < 3; ++cc) {
                if (L) { /* two fluids (nv == NV) */
                    double st[NV][5];
                    int fl[4];
                    for (int v = 0; v < NV; ++v)
                        for (int o = 0; o < 5; ++o) st[v][o] = w7[cc + o][v];
                    learned_cell(g, L, st, lft[cc], rgt[cc], fl, fl + 2);
                } else {
                    for (int v = 0; v < nv; ++v) {
                        double st[5];
                        for (int o = 0; o < 5; ++o) st[o] = w7[cc + o][v];
                        reconstruct_at(g, d, pos[d] - 1 + cc, st, &lft[cc][v], &rgt[cc][v]);
                    }
                }
            }
            double Fm[NVMAX], Fp[NVMAX], um, up;
            hllc(g, rgt[0], lft[1], d, Fm, &um);
            hllc(g, rgt[1], lft[2], d, Fp, &up);
            const double h = cell_width(g, d, pos[d]);
            for (int v = 0; v < nv; ++v) r[v] += (Fm[v] - Fp[v]) / h;
            for (int v = ia0; v < nv; ++v) r[v] += w7[3][v] * ((up - um) / h);
        }
        for (int v = 0; v < nv; ++v) out[c * nv + v] = r[v];
    }
}

void orc_rhs_at(const orc_grid* g, const double* q, int64_t ncell, const int64_t* cells, double* out)
{
    rhs_at_impl(g, q, ncell, cells, out, NULL);
}

/* The learned right-hand side (as orc_rhs_learned, mode 1 per variable, 2
   shared per edge) at selected cells, one by one. */
void orc_rhs_learned_at(const orc_grid* g, const double* q, const double* theta, int mode, int64_t ncell,
                        const int64_t* cells, double* out)
{
    if (nvar(g) != NV) {
        for (int64_t x = 0; x < ncell * nvar(g); ++x) out[x] = NAN;
        return;
    }
    orc_mlp m;
    mlp_load(theta, &m);
    orc_learn L = {&m, mode == 2 ? 2 : 1, 0};
    rhs_at_impl(g, q, ncell, cells, out, &L);
}

/* ---------- CFL time step ---------- */
double orc_cfl_dt(const orc_grid* g, const double* q)
{
    const int64_t N = ncells(g);
    double smax = 0.0;
#pragma omp parallel for reduction(max : smax) schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        const int64_t pos[3] = {c % g->n[0], (c / g->n[0]) % g->n[1], c / ((int64_t)g->n[0] * g->n[1])};
        double qc[NVMAX], wc[NVMAX];
        for (int v = 0; v < nvar(g); ++v) qc[v] = q[v * N + c];
        cons_to_prim(g, qc, wc);
        double cs = sound_speed(g, wc);
        double s = 0.0;
        for (int d = 0; d < 3; ++d)
            if (active(g, d)) s = s + (fabs(wc[imom(g) + d]) + cs) / cell_width(g, d, pos[d]);
        if (s > smax) smax = s;
    }
    return g->cfl / smax;
}

/* ---------- SSP-RK3 (Shu-Osher) ----------
   stage 1: out = qs + dt*L
   stage 2: out = 3/4 qn + 1/4 (qs + dt*L)
   stage 3: out = 1/3 qn + 2/3 (qs + dt*L) */
void orc_rk3_combine(int stage, int64_t n, const double* qn, const double* qs, const double* L,
                     double dt, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < n; ++x) {
        if (stage == 1)
            out[x] = qs[x] + dt * L[x];
        else if (stage == 2)
            out[x] = 0.75 * qn[x] + 0.25 * (qs[x] + dt * L[x]);
        else
            out[x] = (1.0 / 3.0) * qn[x] + (2.0 / 3.0) * (qs[x] + dt * L[x]);
    }
}

/* One SSP-RK3 step in place.  dt <= 0 selects the CFL time step of q.
   Returns the time step used. */
double orc_rk3_step(const orc_grid* g, double* q, double dt)
{
    const int64_t M = nvar(g) * ncells(g);
    if (!(dt > 0.0)) dt = orc_cfl_dt(g, q);
    double* L = (double*)malloc(sizeof(double) * M);
    double* q1 = (double*)malloc(sizeof(double) * M);
    double* q2 = (double*)malloc(sizeof(double) * M);
    orc_rhs(g, q, L);
    orc_rk3_combine(1, M, q, q, L, dt, q1);
    orc_rhs(g, q1, L);
    orc_rk3_combine(2, M, q, q1, L, dt, q2);
    orc_rhs(g, q2, L);
    orc_rk3_combine(3, M, q, q2, L, dt, q);
    free(L);
    free(q1);
    free(q2);
    return dt;
}

/* nsteps steps in place.  dts_in (may be NULL) prescribes each step's dt;
   dts_out (may be NULL) receives the dt used at each step. */
void orc_run(const orc_grid* g, double* q, int nsteps, const double* dts_in, double* dts_out)
{
    for (int s = 0; s < nsteps; ++s) {
        double dt = orc_rk3_step(g, q, dts_in ? dts_in[s] : 0.0);
        if (dts_out) dts_out[s] = dt;
    }
}
