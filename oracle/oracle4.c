/*
 * oracle4.c -- plain, slow FP64 reference for the stencil hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle4.so, which
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load.  It shares no code, header, table or helper with the HIP library and
 * nothing in the HIP library calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no FMA contraction, so every
 * expression below is evaluated exactly as written, in IEEE double).
 *
 * What it computes, with the passage each part follows:
 *
 *   The paper (Cactus/Chemora performance abstractions) describes stencil
 *   loop kernels running over the boxes of a block-structured AMR level with
 *   ghost zones (Sec. II; Sec. III "Loop Traversal"; Sec. IV-D) and prints
 *   only toy stencils: a forward difference and the 2nd-order centred
 *   difference 0.5*(b[i+1]-b[i-1]) (Sec. IV-C3, IV-C4).  The operators here
 *   are the textbook 4th-order centred five-point formulas, the classical
 *   RK4 tableau of Kutta and the discrete adjoint obtained by reverse-mode
 *   differentiation of that RK4 step.  Every discrete operator below IS the
 *   definition of the result; the oracle writes each one out directly.
 *
 * Parity pins (tests that tie this file to mathematics rather than to
 * itself): polynomial exactness with the Taylor defect constants, Fourier
 * symbols, the observed 4th-order convergence rate, the pure-mode RK4 closed
 * form, discrete energy, the adjoint identity, finite-difference gradients
 * and dense-matrix brute force on tiny boxes.
 *
 * Layout of every field of one box: a compact array of
 * (nx+2g)*(ny+2g)*(nz+2g) doubles in C order [z][y][x], x fastest.
 * Interior point (i,j,k), 0 <= i < nx etc., is element
 *   (i+g) + (j+g)*SY + (k+g)*SZ,  SY = nx+2g,  SZ = SY*(ny+2g).
 * Outputs of stencil operators are written on interior points only; their
 * ghost points are left untouched.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int n[3];   /* interior points per axis: x, y, z */
    int g;      /* ghost width */
    long s[3];  /* element strides per axis: 1, SY, SZ */
} grid;

static grid mkgrid(int nx, int ny, int nz, int g)
{
    grid G;
    G.n[0] = nx; G.n[1] = ny; G.n[2] = nz; G.g = g;
    G.s[0] = 1;
    G.s[1] = (long)nx + 2 * g;
    G.s[2] = G.s[1] * ((long)ny + 2 * g);
    return G;
}

static long npoints_total(const grid *G)
{
    return G->s[2] * ((long)G->n[2] + 2 * G->g);
}

/* element index of point (i,j,k); ghost points have coordinates in [-g,0) or [n,n+g) */
static long at(const grid *G, int i, int j, int k)
{
    return (long)(i + G->g) + (long)(j + G->g) * G->s[1] + (long)(k + G->g) * G->s[2];
}

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static double *alloc_field(const grid *G)
{
    return (double *)calloc((size_t)npoints_total(G), sizeof(double));
}

int o4_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the following oracle calls (n >= 1); timing only, results do not depend on it */
void o4_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* --------------------------------------------------------------------------
 * Periodic ghost fill.  Ghost zones hold copies of interior points of the
 * same box, point index taken modulo n (the box is its own periodic
 * neighbour).  Axes are filled in order x, y, z; each later axis copies across
 * the full extent (ghosts included) of the axes already filled, so edges and
 * corners come out right.  In the paper ghost zones are filled by
 * inter-process communication between the bboxes of a level (Sec. II, II-A);
 * a single self-periodic box is the degenerate case.
 */
static void fill_ghosts(const grid *G, double *f)
{
    const int g = G->g, nx = G->n[0], ny = G->n[1], nz = G->n[2];
    int i, j, k;
    /* x faces, over interior y and z */
    for (k = 0; k < nz; k++)
        for (j = 0; j < ny; j++)
            for (i = -g; i < nx + g; i++)
                if (i < 0 || i >= nx)
                    f[at(G, i, j, k)] = f[at(G, wrap(i, nx), j, k)];
    /* y faces, over all x (ghosts included) and interior z */
    for (k = 0; k < nz; k++)
        for (j = -g; j < ny + g; j++)
            if (j < 0 || j >= ny)
                for (i = -g; i < nx + g; i++)
                    f[at(G, i, j, k)] = f[at(G, i, wrap(j, ny), k)];
    /* z faces, over all x and y */
    for (k = -g; k < nz + g; k++)
        if (k < 0 || k >= nz)
            for (j = -g; j < ny + g; j++)
                for (i = -g; i < nx + g; i++)
                    f[at(G, i, j, k)] = f[at(G, i, j, wrap(k, nz))];
}

void o4_fill_ghosts_periodic(int nx, int ny, int nz, int g, double *f)
{
    grid G = mkgrid(nx, ny, nz, g);
    fill_ghosts(&G, f);
}

/* --------------------------------------------------------------------------
 * One-dimensional stencils at a point (textbook 4th-order centred formulas;
 * the paper's own example is the 2nd-order centred difference of Sec. IV-C4):
 *
 *   D1 f_i = ( f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2} ) / (12 h)
 *   D2 f_i = ( -f_{i-2} + 16 f_{i-1} - 30 f_i + 16 f_{i+1} - f_{i+2} ) / (12 h^2)
 *
 * Mixed derivative: the tensor product of two D1 stencils,
 *   D_ab f = sum_{p,q=-2..2} w_p w_q f(x + p e_a + q e_b) / (144 h_a h_b),
 *   w = (1, -8, 0, 8, -1).
 */
static const double W1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
static const double W2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};

static long off(const grid *G, int axis, int p)
{
    return (long)p * G->s[axis];
}

static double pt_d1(const grid *G, const double *f, int axis, double h, long c)
{
    double s = 0.0;
    int p;
    for (p = -2; p <= 2; p++)
        s += W1[p + 2] * f[c + off(G, axis, p)];
    return s / (12.0 * h);
}

static double pt_d2(const grid *G, const double *f, int axis, double h, long c)
{
    double s = 0.0;
    int p;
    for (p = -2; p <= 2; p++)
        s += W2[p + 2] * f[c + off(G, axis, p)];
    return s / (12.0 * h * h);
}

static double pt_dmix(const grid *G, const double *f, int a, int b, double ha, double hb, long c)
{
    double s = 0.0;
    int p, q;
    for (p = -2; p <= 2; p++)
        for (q = -2; q <= 2; q++)
            s += W1[p + 2] * W1[q + 2] * f[c + off(G, a, p) + off(G, b, q)];
    return s / (144.0 * ha * hb);
}

/* Laplacian L f = D2_x f + D2_y f + D2_z f, summed in that order */
static double pt_lap(const grid *G, const double *f, const double dx[3], long c)
{
    return pt_d2(G, f, 0, dx[0], c) + pt_d2(G, f, 1, dx[1], c) + pt_d2(G, f, 2, dx[2], c);
}

void o4_d1(int nx, int ny, int nz, int g, int axis, double h, const double *f, double *out)
{
    grid G = mkgrid(nx, ny, nz, g);
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(&G, i, j, k);
                out[c] = pt_d1(&G, f, axis, h, c);
            }
}

void o4_d2(int nx, int ny, int nz, int g, int axis, double h, const double *f, double *out)
{
    grid G = mkgrid(nx, ny, nz, g);
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(&G, i, j, k);
                out[c] = pt_d2(&G, f, axis, h, c);
            }
}

void o4_dmix(int nx, int ny, int nz, int g, int a, int b, double ha, double hb,
             const double *f, double *out)
{
    grid G = mkgrid(nx, ny, nz, g);
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(&G, i, j, k);
                out[c] = pt_dmix(&G, f, a, b, ha, hb, c);
            }
}

void o4_laplacian(int nx, int ny, int nz, int g, const double dx[3], const double *f, double *out)
{
    grid G = mkgrid(nx, ny, nz, g);
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(&G, i, j, k);
                out[c] = pt_lap(&G, f, dx, c);
            }
}

/* --------------------------------------------------------------------------
 * Scalar wave equation in first-order form, y = (u, rho):
 *   u_t = rho,   rho_t = c^2(x) (L u)(x).
 * The RHS of u is rho itself; this routine returns rho_t only.  c2 == NULL
 * means c = 1.  c2 is read at the point only (never at ghosts).  u's ghosts
 * must already be filled.
 */
void o4_wave_rhs(int nx, int ny, int nz, int g, const double dx[3], const double *u,
                 const double *c2, double *rho_t)
{
    grid G = mkgrid(nx, ny, nz, g);
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(&G, i, j, k);
                double lu = pt_lap(&G, u, dx, c);
                rho_t[c] = c2 ? c2[c] * lu : lu;
            }
}

/* F(y) for the RK4 stages: fills u's ghosts periodically, then
 * ku = rho, kr = c^2 L u on interior points. */
static void wave_F(const grid *G, const double dx[3], const double *c2, double *u,
                   const double *rho, double *ku, double *kr)
{
    const int nx = G->n[0], ny = G->n[1], nz = G->n[2];
    int k;
    fill_ghosts(G, u);
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(G, i, j, k);
                double lu = pt_lap(G, u, dx, c);
                ku[c] = rho[c];
                kr[c] = c2 ? c2[c] * lu : lu;
            }
}

/* y_s = y_n + a * k on interior points */
static void axpy_interior(const grid *G, double a, const double *yn, const double *kk, double *ys)
{
    const int nx = G->n[0], ny = G->n[1], nz = G->n[2];
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(G, i, j, k);
                ys[c] = yn[c] + a * kk[c];
            }
}

/*
 * Classical RK4 (Kutta):
 *   k1 = F(y_n)
 *   k2 = F(y_n + dt/2 k1)
 *   k3 = F(y_n + dt/2 k2)
 *   k4 = F(y_n + dt   k3)
 *   y_{n+1} = y_n + dt/6 (k1 + 2 k2 + 2 k3 + k4)
 * with a periodic ghost fill of the stage u before every F.  Advances (u, rho)
 * in place by nsteps steps; u's ghosts are overwritten by the fills.
 */
void o4_rk4(int nx, int ny, int nz, int g, const double dx[3], const double *c2, double dt,
            int nsteps, double *u, double *rho)
{
    grid G = mkgrid(nx, ny, nz, g);
    double *ku[4], *kr[4], *su = alloc_field(&G), *sr = alloc_field(&G);
    int s, step, k;
    for (s = 0; s < 4; s++) {
        ku[s] = alloc_field(&G);
        kr[s] = alloc_field(&G);
    }
    for (step = 0; step < nsteps; step++) {
        wave_F(&G, dx, c2, u, rho, ku[0], kr[0]);
        axpy_interior(&G, 0.5 * dt, u, ku[0], su);
        axpy_interior(&G, 0.5 * dt, rho, kr[0], sr);
        wave_F(&G, dx, c2, su, sr, ku[1], kr[1]);
        axpy_interior(&G, 0.5 * dt, u, ku[1], su);
        axpy_interior(&G, 0.5 * dt, rho, kr[1], sr);
        wave_F(&G, dx, c2, su, sr, ku[2], kr[2]);
        axpy_interior(&G, dt, u, ku[2], su);
        axpy_interior(&G, dt, rho, kr[2], sr);
        wave_F(&G, dx, c2, su, sr, ku[3], kr[3]);
#pragma omp parallel for schedule(static)
        for (k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    long c = at(&G, i, j, k);
                    u[c] = u[c] + dt / 6.0 * (ku[0][c] + 2.0 * ku[1][c] + 2.0 * ku[2][c] + ku[3][c]);
                    rho[c] = rho[c] + dt / 6.0 * (kr[0][c] + 2.0 * kr[1][c] + 2.0 * kr[2][c] + kr[3][c]);
                }
    }
    for (s = 0; s < 4; s++) {
        free(ku[s]);
        free(kr[s]);
    }
    free(su);
    free(sr);
}

/* --------------------------------------------------------------------------
 * Multi-field derivative kernel, for one field f (each output depends on its
 * own input only):
 *   out = sum_a D2_a f + sum_{a<b} D_ab f + sum_{a,b} A[a][b] (D1_a f)(D1_b f)
 * with axes a, b in {x, y, z} = {0, 1, 2} and A a 3x3 row-major matrix
 * (symmetric in the workloads, but used here exactly as given).  f's ghosts
 * (edges included, which the mixed terms read) must already be filled.
 */
void o4_deriv_mixed(int nx, int ny, int nz, int g, const double dx[3], const double A[9],
                    const double *f, double *out)
{
    grid G = mkgrid(nx, ny, nz, g);
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(&G, i, j, k);
                double d1[3], s = 0.0;
                int a, b;
                for (a = 0; a < 3; a++)
                    s += pt_d2(&G, f, a, dx[a], c);
                for (a = 0; a < 3; a++)
                    for (b = a + 1; b < 3; b++)
                        s += pt_dmix(&G, f, a, b, dx[a], dx[b], c);
                for (a = 0; a < 3; a++)
                    d1[a] = pt_d1(&G, f, a, dx[a], c);
                for (a = 0; a < 3; a++)
                    for (b = 0; b < 3; b++)
                        s += A[3 * a + b] * d1[a] * d1[b];
                out[c] = s;
            }
}

/* --------------------------------------------------------------------------
 * Adjoint of the wave RHS.  As a linear map of interior values,
 *   F(u, rho) = (rho, C L_p u),   C = diag(c^2),
 * where L_p is "periodic ghost fill, then the Laplacian stencil".  L_p is a
 * symmetric circulant, so
 *   F^T(lu, lrho) = (L_p (C lrho), lu):
 * form w = c^2 * lrho on the interior, fill w's ghosts periodically, apply L.
 * This identity holds only for periodic boxes.  c2 == NULL means c = 1.
 */
static void wave_FT(const grid *G, const double dx[3], const double *c2, const double *lu,
                    const double *lrho, double *w, double *out_u, double *out_rho)
{
    const int nx = G->n[0], ny = G->n[1], nz = G->n[2];
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(G, i, j, k);
                w[c] = c2 ? c2[c] * lrho[c] : lrho[c];
            }
    fill_ghosts(G, w);
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(G, i, j, k);
                out_u[c] = pt_lap(G, w, dx, c);
                out_rho[c] = lu[c];
            }
}

void o4_wave_adjoint_rhs(int nx, int ny, int nz, int g, const double dx[3], const double *lu,
                         const double *lrho, const double *c2, double *out_u, double *out_rho)
{
    grid G = mkgrid(nx, ny, nz, g);
    double *w = alloc_field(&G);
    wave_FT(&G, dx, c2, lu, lrho, w, out_u, out_rho);
    free(w);
}

/*
 * One backward RK4 step (reverse-mode differentiation of o4_rk4's step).
 *
 * Forward step from y_n (stage inputs y_1 = y_n, y_2, y_3, y_4):
 *   k_s = F(y_s);  y_2 = y_n + dt/2 k1;  y_3 = y_n + dt/2 k2;  y_4 = y_n + dt k3;
 *   y_{n+1} = y_n + dt/6 (k1 + 2 k2 + 2 k3 + k4).
 * Given ybar = dJ/dy_{n+1} (lam_u, lam_rho), walking the statements backwards:
 *   kb4 = dt/6 ybar                 ; yb4 = F^T kb4
 *   kb3 = dt/3 ybar + dt   yb4      ; yb3 = F^T kb3
 *   kb2 = dt/3 ybar + dt/2 yb3      ; yb2 = F^T kb2
 *   kb1 = dt/6 ybar + dt/2 yb2      ; yb1 = F^T kb1
 *   ybar_n = ybar + yb1 + yb2 + yb3 + yb4
 * and, because k_s's rho part is c^2 * (L_p u_s),
 *   c2bar += sum_s (kb_s)_rho * (L_p u_s).
 * u_n and rho_n are the forward state at the start of the step; the stage
 * states are recomputed here.  lam_u, lam_rho are overwritten with ybar_n;
 * c2bar is accumulated into (interior points).  c2 == NULL means c = 1 (then
 * c2bar may be NULL).  u_n and rho_n are not modified.
 */
static void rk4_adjoint_step(const grid *G, const double dx[3], const double *c2, double dt,
                             const double *u_n, const double *rho_n, double *lam_u, double *lam_rho,
                             double *c2bar)
{
    const int nx = G->n[0], ny = G->n[1], nz = G->n[2];
    double *us[4], *rs = alloc_field(G), *ku = alloc_field(G), *kr = alloc_field(G);
    double *kbu = alloc_field(G), *kbr = alloc_field(G), *w = alloc_field(G);
    double *ybu[4], *ybr[4], *lus = alloc_field(G);
    int s, k;
    static const double cstage[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}; /* weight of k_s in y_{n+1} */
    static const double astage[4] = {0.5, 0.5, 1.0, 0.0}; /* y_{s+1} = y_n + a_s dt k_s */

    for (s = 0; s < 4; s++) {
        us[s] = alloc_field(G);
        ybu[s] = alloc_field(G);
        ybr[s] = alloc_field(G);
    }
    /* forward recompute of the stage states u_1..u_4 (rho only needed transiently) */
    memcpy(us[0], u_n, sizeof(double) * (size_t)npoints_total(G));
    memcpy(rs, rho_n, sizeof(double) * (size_t)npoints_total(G));
    for (s = 0; s < 3; s++) {
        wave_F(G, dx, c2, us[s], rs, ku, kr); /* fills us[s]'s ghosts */
        axpy_interior(G, astage[s] * dt, u_n, ku, us[s + 1]);
        axpy_interior(G, astage[s] * dt, rho_n, kr, rs);
    }
    fill_ghosts(G, us[3]);

    /* reverse sweep, s = 4, 3, 2, 1 (index 3..0) */
    for (s = 3; s >= 0; s--) {
#pragma omp parallel for schedule(static)
        for (k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    long c = at(G, i, j, k);
                    double bu = cstage[s] * dt * lam_u[c];
                    double br = cstage[s] * dt * lam_rho[c];
                    if (s < 3) { /* y_{s+1} = y_n + a_s dt k_s */
                        bu += astage[s] * dt * ybu[s + 1][c];
                        br += astage[s] * dt * ybr[s + 1][c];
                    }
                    kbu[c] = bu;
                    kbr[c] = br;
                }
        wave_FT(G, dx, c2, kbu, kbr, w, ybu[s], ybr[s]);
        if (c2bar) {
#pragma omp parallel for schedule(static)
            for (k = 0; k < nz; k++)
                for (int j = 0; j < ny; j++)
                    for (int i = 0; i < nx; i++) {
                        long c = at(G, i, j, k);
                        lus[c] = pt_lap(G, us[s], dx, c);
                        c2bar[c] += kbr[c] * lus[c];
                    }
        }
    }
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(G, i, j, k);
                lam_u[c] = lam_u[c] + ybu[0][c] + ybu[1][c] + ybu[2][c] + ybu[3][c];
                lam_rho[c] = lam_rho[c] + ybr[0][c] + ybr[1][c] + ybr[2][c] + ybr[3][c];
            }
    for (s = 0; s < 4; s++) {
        free(us[s]);
        free(ybu[s]);
        free(ybr[s]);
    }
    free(rs); free(ku); free(kr); free(kbu); free(kbr); free(w); free(lus);
}

void o4_rk4_adjoint_step(int nx, int ny, int nz, int g, const double dx[3], const double *c2,
                         double dt, const double *u_n, const double *rho_n, double *lam_u,
                         double *lam_rho, double *c2bar)
{
    grid G = mkgrid(nx, ny, nz, g);
    rk4_adjoint_step(&G, dx, c2, dt, u_n, rho_n, lam_u, lam_rho, c2bar);
}

/*
 * Loss and gradient, store-all (no checkpointing):
 *   J = 1/2 sum_{interior} (u_N - u_target)^2,  N = nsteps,
 * with u_N from o4_rk4 started at (u0, rho0).  Returns J and writes
 * dJ/du0, dJ/drho0 and dJ/dc2 (interior points; ghosts zero).  The sum is
 * taken serially in C order.  Every forward state is kept (2*(nsteps+1)
 * fields) and the backward steps run from N-1 down to 0.
 */
double o4_wave_loss_grad(int nx, int ny, int nz, int g, const double dx[3], const double *c2,
                         double dt, int nsteps, const double *u0, const double *rho0,
                         const double *u_target, double *ubar0, double *rhobar0, double *c2bar)
{
    grid G = mkgrid(nx, ny, nz, g);
    size_t bytes = sizeof(double) * (size_t)npoints_total(&G);
    if (nsteps < 0)
        return NAN;
    double **U = (double **)malloc(sizeof(double *) * (size_t)(nsteps + 1));
    double **R = (double **)malloc(sizeof(double *) * (size_t)(nsteps + 1));
    double J = 0.0;
    int n;
    for (n = 0; n <= nsteps; n++) {
        U[n] = alloc_field(&G);
        R[n] = alloc_field(&G);
    }
    memcpy(U[0], u0, bytes);
    memcpy(R[0], rho0, bytes);
    for (n = 0; n < nsteps; n++) {
        memcpy(U[n + 1], U[n], bytes);
        memcpy(R[n + 1], R[n], bytes);
        o4_rk4(nx, ny, nz, g, dx, c2, dt, 1, U[n + 1], R[n + 1]);
    }
    memset(ubar0, 0, bytes);
    memset(rhobar0, 0, bytes);
    if (c2bar)
        memset(c2bar, 0, bytes);
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                long c = at(&G, i, j, k);
                double d = U[nsteps][c] - u_target[c];
                J += 0.5 * d * d;
                ubar0[c] = d;
            }
    for (n = nsteps - 1; n >= 0; n--)
        rk4_adjoint_step(&G, dx, c2, dt, U[n], R[n], ubar0, rhobar0, c2bar);
    for (n = 0; n <= nsteps; n++) {
        free(U[n]);
        free(R[n]);
    }
    free(U);
    free(R);
    return J;
}
