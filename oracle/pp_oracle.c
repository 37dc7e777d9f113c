/*
 * pp_oracle.c -- plain FP64 CPU oracle for the pressure-projection step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code with
 * the HIP path; it is written for obviousness, not speed (plain loops over
 * cells, OpenMP only around independent per-cell work).
 *
 * What it computes (paper Sec. 3.1-3.2, Sec. 3.7.1, Sec. 3.8):
 *   - staggered (MAC) grid, cubic cells of edge h; p at cell centres, the
 *     normal velocity u_m on the faces (Sec. 3.1, eqs. cont2 / incompdisc3);
 *   - face coefficients beta = 1/rho interpolated from the two neighbouring
 *     cells (Sec. 3.7.1: coefficients are interpolations of 1/rho); we take
 *     beta = 2 / (rho_L + rho_R), i.e. arithmetic averaging of rho;
 *   - the discrete divergence D u (eq. cont2);
 *   - the pressure operator A p = D (beta G p), whose coefficients satisfy
 *     A7 = sum A1..A6 and A2_i = A1_{i+1} etc. (Sec. 3.7.1);
 *   - the projection u = u* - dt beta G p (eq. fotm) with p solving
 *     A p = D u* / dt (eq. poisson, with the time step moved to the right);
 *   - walls: Neumann for p by zeroing the coefficient of a wall link
 *     (Sec. 3.8), and zero normal velocity on wall faces;
 *   - the paper's red-black Gauss-Seidel with over-relaxation
 *     (Sec. 3.7.1, eq. beta_pressure), used as a cross-check;
 *   - the adjoint of the solve: dL/d rhs and dL/d beta for L = <w, p>;
 *   - a general operator A - diag(sigma) with closed interior links (solid
 *     link flags, Sec. 3.8), a diagonal term (the implicit viscous step,
 *     Sec. 3.2.3; free-surface Dirichlet branches, Sec. 3.7.5) and excluded
 *     cells, solved by Jacobi-preconditioned conjugate gradients.
 *
 * Layout: cell arrays (nz, ny, nx), C order, x fastest.  A face array for
 * direction m has the same shape; entry c is the LOW face of cell c in
 * direction m.  In a wall direction the entry with c_m == 0 is the wall face
 * (its stored value is ignored and treated as zero); the upper wall face is
 * implicit.  In a periodic direction c - e_m wraps around.
 *
 * The operator is singular (constants are in its null space for periodic and
 * walled boxes).  The solve removes the mean of the right-hand side and
 * returns the mean-zero solution.  Readings where the paper is silent:
 *   - index pairing of eq. beta_pressure: A5 <-> k-1 and A6 <-> k+1, which
 *     is what the coefficient relation A6_k = A5_{k+1} requires;
 *   - the solver for grids above a few thousand cells is conjugate
 *     gradients preconditioned by a symmetric multigrid V-cycle (damped
 *     Jacobi smoothing, trilinear prolongation, its transpose as
 *     restriction, coarse beta = mean of the four sub-faces, dense coarsest
 *     solve); only its converged answer matters, not its iterates.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n[3];   /* nx, ny, nz */
    int bc[3];      /* 0 periodic, 1 wall */
    double h;
} grid_t;

static int64_t cells(const grid_t *g) { return g->n[0] * g->n[1] * g->n[2]; }

static int64_t lin(const grid_t *g, int64_t i, int64_t j, int64_t k)
{
    return (k * g->n[1] + j) * g->n[0] + i;
}

/* coordinates of cell c as (i, j, k) */
static void coords(const grid_t *g, int64_t c, int64_t ijk[3])
{
    ijk[0] = c % g->n[0];
    ijk[1] = (c / g->n[0]) % g->n[1];
    ijk[2] = c / (g->n[0] * g->n[1]);
}

/* neighbour of cell ijk in direction m, offset s = -1 or +1, with periodic
 * wrap.  Returns -1 when the step would cross a wall. */
static int64_t neighbour(const grid_t *g, const int64_t ijk[3], int m, int s)
{
    int64_t q[3] = {ijk[0], ijk[1], ijk[2]};
    q[m] += s;
    if (q[m] < 0 || q[m] >= g->n[m]) {
        if (g->bc[m] == 1)
            return -1;
        q[m] = (q[m] + g->n[m]) % g->n[m];
    }
    return lin(g, q[0], q[1], q[2]);
}

/* beta of the low face of cell ijk in direction m (0 at a wall) */
static double beta_low(const grid_t *g, const double *const beta[3], const int64_t ijk[3], int m)
{
    if (g->bc[m] == 1 && ijk[m] == 0)
        return 0.0;
    return beta[m][lin(g, ijk[0], ijk[1], ijk[2])];
}

/* beta of the high face of cell ijk in direction m (0 at a wall) */
static double beta_high(const grid_t *g, const double *const beta[3], const int64_t ijk[3], int m)
{
    int64_t up = neighbour(g, ijk, m, +1);
    if (up < 0)
        return 0.0;
    return beta[m][up];
}

static grid_t make_grid(const int64_t *n, const int *bc, double h)
{
    grid_t g;
    for (int m = 0; m < 3; ++m) {
        g.n[m] = n[m];
        g.bc[m] = bc[m];
    }
    g.h = h;
    return g;
}

/* number of threads the parallel loops use */
EXPORT int ppo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* number of threads later parallel loops of the calling thread use (n >= 1);
   for timing only: sums over cells may then group their terms differently */
EXPORT void ppo_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* face coefficients, divergence, operator, projection                       */
/* ------------------------------------------------------------------------ */

/* beta_m[c] = 2 / (rho[c - e_m] + rho[c]) on every non-wall face, 0 on walls. */
EXPORT void ppo_face_coeffs(const int64_t *n, const int *bc, const double *rho,
                            double *bx, double *by, double *bz)
{
    grid_t g = make_grid(n, bc, 1.0);
    double *beta[3] = {bx, by, bz};
    int64_t N = cells(&g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(&g, c, ijk);
        for (int m = 0; m < 3; ++m) {
            int64_t lo = neighbour(&g, ijk, m, -1);
            beta[m][c] = (lo < 0) ? 0.0 : 2.0 / (rho[lo] + rho[c]);
        }
    }
}

/* out[c] = scale * sum_m (u_m(high face) - u_m(low face)) / h, wall faces 0
 * (eq. cont2). */
EXPORT void ppo_divergence(const int64_t *n, const int *bc, double h, const double *ux,
                           const double *uy, const double *uz, double scale, double *out)
{
    grid_t g = make_grid(n, bc, h);
    const double *u[3] = {ux, uy, uz};
    int64_t N = cells(&g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(&g, c, ijk);
        double s = 0.0;
        for (int m = 0; m < 3; ++m) {
            double lo = (g.bc[m] == 1 && ijk[m] == 0) ? 0.0 : u[m][c];
            int64_t up = neighbour(&g, ijk, m, +1);
            double hi = (up < 0) ? 0.0 : u[m][up];
            s += (hi - lo) / h;
        }
        out[c] = scale * s;
    }
}

/* y = A x with (A x)[c] = sum_m [beta_hi (x_up - x_c) - beta_lo (x_c - x_dn)] / h^2 */
static void apply_A(const grid_t *g, const double *const beta[3], const double *x, double *y)
{
    int64_t N = cells(g);
    double ih2 = 1.0 / (g->h * g->h);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(g, c, ijk);
        double s = 0.0;
        for (int m = 0; m < 3; ++m) {
            int64_t dn = neighbour(g, ijk, m, -1);
            int64_t up = neighbour(g, ijk, m, +1);
            if (up >= 0)
                s += beta_high(g, beta, ijk, m) * (x[up] - x[c]);
            if (dn >= 0)
                s -= beta_low(g, beta, ijk, m) * (x[c] - x[dn]);
        }
        y[c] = s * ih2;
    }
}

EXPORT void ppo_apply(const int64_t *n, const int *bc, double h, const double *bx,
                      const double *by, const double *bz, const double *x, double *y)
{
    grid_t g = make_grid(n, bc, h);
    const double *beta[3] = {bx, by, bz};
    apply_A(&g, beta, x, y);
}

/* u_m[c] = u*_m[c] - dt * beta_m[c] * (p[c] - p[c - e_m]) / h on non-wall
 * faces, 0 on wall faces (eq. fotm; link masks of Sec. 3.8). */
EXPORT void ppo_project(const int64_t *n, const int *bc, double h, double dt, const double *bx,
                        const double *by, const double *bz, const double *usx,
                        const double *usy, const double *usz, const double *p, double *ux,
                        double *uy, double *uz)
{
    grid_t g = make_grid(n, bc, h);
    const double *beta[3] = {bx, by, bz};
    const double *us[3] = {usx, usy, usz};
    double *u[3] = {ux, uy, uz};
    int64_t N = cells(&g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(&g, c, ijk);
        for (int m = 0; m < 3; ++m) {
            int64_t dn = neighbour(&g, ijk, m, -1);
            if (dn < 0) {
                u[m][c] = 0.0;
                continue;
            }
            double grad = (p[c] - p[dn]) / h;
            u[m][c] = us[m][c] - dt * beta[m][c] * grad;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* the paper's red-black Gauss-Seidel with over-relaxation (eq. beta_pressure) */
/* ------------------------------------------------------------------------ */

/* One colour pass of eq. beta_pressure: A1..A6 are the six link coefficients
 * (beta of the face / h^2), A7 their sum, A8 the right-hand side. */
static void sor_colour(const grid_t *g, const double *const beta[3], const double *rhs,
                       double *p, double omega, int colour)
{
    int64_t N = cells(g);
    double ih2 = 1.0 / (g->h * g->h);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(g, c, ijk);
        if (((ijk[0] + ijk[1] + ijk[2]) & 1) != colour)
            continue;
        int64_t nb[6];
        double A[7];
        /* A1: i-1, A2: i+1, A3: j-1, A4: j+1, A5: k-1, A6: k+1 */
        for (int m = 0; m < 3; ++m) {
            nb[2 * m] = neighbour(g, ijk, m, -1);
            nb[2 * m + 1] = neighbour(g, ijk, m, +1);
            A[2 * m] = beta_low(g, beta, ijk, m) * ih2;
            A[2 * m + 1] = beta_high(g, beta, ijk, m) * ih2;
        }
        double A7 = 0.0, sum = 0.0;
        for (int q = 0; q < 6; ++q) {
            A7 += A[q];
            if (nb[q] >= 0)
                sum += A[q] * p[nb[q]];
        }
        double A8 = rhs[c];
        p[c] = (1.0 - omega) * p[c] + (omega / A7) * (sum - A8);
    }
}

static double norm2(const double *x, int64_t N)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t c = 0; c < N; ++c)
        s += x[c] * x[c];
    return sqrt(s);
}

/* Red (i+j+k even) first, then black (first = 0; the paper's order), or
 * black first (first = 1), `sweeps` times or until the relative L2 residual
 * ||rhs - A p|| / ||rhs|| <= tol (checked after each sweep when tol > 0).
 * rhs is used as given (no mean removal); p is updated in place.  Returns
 * the number of sweeps done; *relres receives the last residual. */
EXPORT int ppo_rbsor(const int64_t *n, const int *bc, double h, const double *bx,
                     const double *by, const double *bz, const double *rhs, double *p,
                     double omega, int sweeps, double tol, int first, double *relres)
{
    grid_t g = make_grid(n, bc, h);
    const double *beta[3] = {bx, by, bz};
    int64_t N = cells(&g);
    double *r = (double *)malloc(sizeof(double) * N);
    double nb = norm2(rhs, N);
    int s = 0;
    double rel = 0.0;
    for (s = 0; s < sweeps;) {
        sor_colour(&g, beta, rhs, p, omega, first);
        sor_colour(&g, beta, rhs, p, omega, 1 - first);
        ++s;
        if (tol > 0.0) {
            apply_A(&g, beta, p, r);
            for (int64_t c = 0; c < N; ++c)
                r[c] = rhs[c] - r[c];
            rel = norm2(r, N) / (nb > 0 ? nb : 1.0);
            if (rel <= tol)
                break;
        }
    }
    if (relres) {
        apply_A(&g, beta, p, r);
        for (int64_t c = 0; c < N; ++c)
            r[c] = rhs[c] - r[c];
        *relres = norm2(r, N) / (nb > 0 ? nb : 1.0);
    }
    free(r);
    return s;
}

/* ------------------------------------------------------------------------ */
/* multigrid-preconditioned conjugate gradients                              */
/* ------------------------------------------------------------------------ */

#define MAXLEV 24
#define COARSEST_MAX 512

typedef struct {
    grid_t g;
    double *beta[3];
    double *diag;            /* sum of the six link coefficients (>= 0) */
    double *x, *b, *t;       /* work vectors on this level */
    /* per-axis prolongation tables (fine index -> parent, other, weights) */
    int64_t *par[3], *oth[3];
    /* per-axis restriction tables in CSR form (coarse index -> fine list) */
    int64_t *rptr[3], *ridx[3];
    double *rw[3];
} level_t;

typedef struct {
    int nlev;
    level_t L[MAXLEV];
    double *chol;            /* Cholesky factor of the coarsest shifted operator */
    int64_t nc;
} mg_t;

static void compute_diag(level_t *lv)
{
    grid_t *g = &lv->g;
    int64_t N = cells(g);
    double ih2 = 1.0 / (g->h * g->h);
    const double *beta[3] = {lv->beta[0], lv->beta[1], lv->beta[2]};
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(g, c, ijk);
        double d = 0.0;
        for (int m = 0; m < 3; ++m)
            d += beta_low(g, beta, ijk, m) + beta_high(g, beta, ijk, m);
        lv->diag[c] = d * ih2;
    }
}

/* Cell-centred linear interpolation along one axis: fine cell i takes 3/4 of
 * its parent i/2 and 1/4 of the next coarse cell on its side; at a wall the
 * missing coarse cell is replaced by the parent itself. */
static void build_axis_tables(level_t *fine, int m, int64_t nH)
{
    int64_t nh = fine->g.n[m];
    fine->par[m] = (int64_t *)malloc(sizeof(int64_t) * nh);
    fine->oth[m] = (int64_t *)malloc(sizeof(int64_t) * nh);
    for (int64_t i = 0; i < nh; ++i) {
        int64_t I = i / 2;
        int64_t O = (i % 2 == 0) ? I - 1 : I + 1;
        if (O < 0 || O >= nH) {
            if (fine->g.bc[m] == 1)
                O = I;
            else
                O = (O + nH) % nH;
        }
        fine->par[m][i] = I;
        fine->oth[m][i] = O;
    }
    /* the transpose, gathered per coarse index */
    int64_t *cnt = (int64_t *)calloc(nH + 1, sizeof(int64_t));
    for (int64_t i = 0; i < nh; ++i) {
        cnt[fine->par[m][i] + 1]++;
        cnt[fine->oth[m][i] + 1]++;
    }
    for (int64_t I = 0; I < nH; ++I)
        cnt[I + 1] += cnt[I];
    fine->rptr[m] = cnt;
    fine->ridx[m] = (int64_t *)malloc(sizeof(int64_t) * 2 * nh);
    fine->rw[m] = (double *)malloc(sizeof(double) * 2 * nh);
    int64_t *fill = (int64_t *)calloc(nH, sizeof(int64_t));
    for (int64_t i = 0; i < nh; ++i) {
        int64_t I = fine->par[m][i], O = fine->oth[m][i];
        int64_t a = cnt[I] + fill[I]++;
        fine->ridx[m][a] = i;
        fine->rw[m][a] = 0.75;
        int64_t b = cnt[O] + fill[O]++;
        fine->ridx[m][b] = i;
        fine->rw[m][b] = 0.25;
    }
    free(fill);
}

/* fine x += P xH */
static void prolong_add(const level_t *fine, const level_t *coarse, const double *xH, double *x)
{
    const grid_t *g = &fine->g;
    int64_t N = cells(g);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(g, c, ijk);
        int64_t ci[2] = {fine->par[0][ijk[0]], fine->oth[0][ijk[0]]};
        int64_t cj[2] = {fine->par[1][ijk[1]], fine->oth[1][ijk[1]]};
        int64_t ck[2] = {fine->par[2][ijk[2]], fine->oth[2][ijk[2]]};
        const double w[2] = {0.75, 0.25};
        double s = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d)
                    s += w[a] * w[b] * w[d] * xH[lin(&coarse->g, ci[d], cj[b], ck[a])];
        x[c] += s;
    }
}

/* bH = (1/8) P^T r */
static void restrict_T(const level_t *fine, const level_t *coarse, const double *r, double *bH)
{
    const grid_t *G = &coarse->g;
    int64_t N = cells(G);
#pragma omp parallel for schedule(static)
    for (int64_t C = 0; C < N; ++C) {
        int64_t IJK[3];
        coords(G, C, IJK);
        double s = 0.0;
        for (int64_t a = fine->rptr[2][IJK[2]]; a < fine->rptr[2][IJK[2] + 1]; ++a)
            for (int64_t b = fine->rptr[1][IJK[1]]; b < fine->rptr[1][IJK[1] + 1]; ++b)
                for (int64_t d = fine->rptr[0][IJK[0]]; d < fine->rptr[0][IJK[0] + 1]; ++d)
                    s += fine->rw[2][a] * fine->rw[1][b] * fine->rw[0][d] *
                         r[lin(&fine->g, fine->ridx[0][d], fine->ridx[1][b], fine->ridx[2][a])];
        bH[C] = s / 8.0;
    }
}

/* coarse beta = mean of the four fine faces that make up each coarse face */
static void coarsen_beta(const level_t *fine, level_t *coarse)
{
    const grid_t *G = &coarse->g;
    int64_t N = cells(G);
    for (int m = 0; m < 3; ++m) {
#pragma omp parallel for schedule(static)
        for (int64_t C = 0; C < N; ++C) {
            int64_t IJK[3];
            coords(G, C, IJK);
            double s = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    int64_t f[3] = {2 * IJK[0], 2 * IJK[1], 2 * IJK[2]};
                    int t1 = (m + 1) % 3, t2 = (m + 2) % 3;
                    f[t1] += a;
                    f[t2] += b;
                    if (fine->g.bc[m] == 1 && f[m] == 0)
                        continue;
                    s += fine->beta[m][lin(&fine->g, f[0], f[1], f[2])];
                }
            coarse->beta[m][C] = s / 4.0;
        }
    }
}

static int cholesky(double *a, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = a[j * n + j];
        for (int64_t k = 0; k < j; ++k)
            d -= a[j * n + k] * a[j * n + k];
        if (!(d > 0.0))
            return -1;
        d = sqrt(d);
        a[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = a[i * n + j];
            for (int64_t k = 0; k < j; ++k)
                s -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = s / d;
        }
    }
    return 0;
}

/* Coarsest level: factor K = -A + (s/n) 1 1^T, which is positive definite
 * on a connected grid; K e = -r with mean(r) = 0 gives A e = r, mean(e) = 0. */
static int build_coarsest(mg_t *mg)
{
    level_t *lv = &mg->L[mg->nlev - 1];
    int64_t n = cells(&lv->g);
    double *K = (double *)calloc(n * n, sizeof(double));
    double *e = (double *)calloc(n, sizeof(double));
    double *col = (double *)calloc(n, sizeof(double));
    const double *beta[3] = {lv->beta[0], lv->beta[1], lv->beta[2]};
    double smax = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        memset(e, 0, sizeof(double) * n);
        e[j] = 1.0;
        apply_A(&lv->g, beta, e, col);
        for (int64_t i = 0; i < n; ++i)
            K[i * n + j] = -col[i];
        if (-col[j] > smax)
            smax = -col[j];
    }
    for (int64_t i = 0; i < n * n; ++i)
        K[i] += smax / (double)n;
    int rc = cholesky(K, n);
    mg->chol = K;
    mg->nc = n;
    free(e);
    free(col);
    return rc;
}

static void coarsest_solve(const mg_t *mg, const double *r, double *x)
{
    int64_t n = mg->nc;
    const double *L = mg->chol;
    double mean = 0.0;
    for (int64_t i = 0; i < n; ++i)
        mean += r[i];
    mean /= (double)n;
    /* forward: L y = -(r - mean) */
    for (int64_t i = 0; i < n; ++i) {
        double s = -(r[i] - mean);
        for (int64_t k = 0; k < i; ++k)
            s -= L[i * n + k] * x[k];
        x[i] = s / L[i * n + i];
    }
    /* backward: L^T x = y */
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int64_t k = i + 1; k < n; ++k)
            s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
}

static void mg_free(mg_t *mg)
{
    for (int l = 0; l < mg->nlev; ++l) {
        level_t *lv = &mg->L[l];
        for (int m = 0; m < 3; ++m) {
            if (l > 0)
                free(lv->beta[m]);
            free(lv->par[m]);
            free(lv->oth[m]);
            free(lv->rptr[m]);
            free(lv->ridx[m]);
            free(lv->rw[m]);
        }
        free(lv->diag);
        free(lv->x);
        free(lv->b);
        free(lv->t);
    }
    free(mg->chol);
}

static int mg_build(mg_t *mg, const grid_t *g, const double *const beta[3])
{
    memset(mg, 0, sizeof(*mg));
    mg->L[0].g = *g;
    for (int m = 0; m < 3; ++m)
        mg->L[0].beta[m] = (double *)beta[m];
    int l = 0;
    for (;;) {
        level_t *lv = &mg->L[l];
        int64_t N = cells(&lv->g);
        lv->diag = (double *)malloc(sizeof(double) * N);
        lv->x = (double *)calloc(N, sizeof(double));
        lv->b = (double *)calloc(N, sizeof(double));
        lv->t = (double *)calloc(N, sizeof(double));
        compute_diag(lv);
        int can = N > COARSEST_MAX && l + 1 < MAXLEV;
        for (int m = 0; m < 3; ++m)
            can = can && (lv->g.n[m] % 2 == 0) && (lv->g.n[m] >= 4);
        if (!can)
            break;
        level_t *cv = &mg->L[l + 1];
        cv->g = lv->g;
        for (int m = 0; m < 3; ++m)
            cv->g.n[m] = lv->g.n[m] / 2;
        cv->g.h = 2.0 * lv->g.h;
        int64_t NC = cells(&cv->g);
        for (int m = 0; m < 3; ++m) {
            cv->beta[m] = (double *)malloc(sizeof(double) * NC);
            build_axis_tables(lv, m, cv->g.n[m]);
        }
        coarsen_beta(lv, cv);
        ++l;
    }
    mg->nlev = l + 1;
    if (cells(&mg->L[l].g) > 4096)
        return -2;
    return build_coarsest(mg);
}

/* damped Jacobi: x += omega D^-1 (b - A x); symmetric as a smoother */
static void jacobi(level_t *lv, const double *b, double *x, int sweeps)
{
    const double *beta[3] = {lv->beta[0], lv->beta[1], lv->beta[2]};
    int64_t N = cells(&lv->g);
    const double omega = 0.8;
    for (int s = 0; s < sweeps; ++s) {
        apply_A(&lv->g, beta, x, lv->t);
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < N; ++c)
            x[c] -= omega * (b[c] - lv->t[c]) / lv->diag[c];
    }
}

/* One V-cycle for A x = b starting from x = 0; symmetric in b -> x. */
static void vcycle(mg_t *mg, int l, const double *b, double *x)
{
    level_t *lv = &mg->L[l];
    int64_t N = cells(&lv->g);
    if (l == mg->nlev - 1) {
        coarsest_solve(mg, b, x);
        return;
    }
    memset(x, 0, sizeof(double) * N);
    /* A is negative semi-definite; the Jacobi update above uses -D, so the
     * sign convention is x -= omega (b - A x) / diag with diag = -A_cc. */
    jacobi(lv, b, x, 2);
    const double *beta[3] = {lv->beta[0], lv->beta[1], lv->beta[2]};
    apply_A(&lv->g, beta, x, lv->t);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c)
        lv->t[c] = b[c] - lv->t[c];
    level_t *cv = &mg->L[l + 1];
    restrict_T(lv, cv, lv->t, cv->b);
    vcycle(mg, l + 1, cv->b, cv->x);
    prolong_add(lv, cv, cv->x, x);
    jacobi(lv, b, x, 2);
}

static void remove_mean(double *x, int64_t N)
{
    double s = 0.0;
    for (int64_t c = 0; c < N; ++c)
        s += x[c];
    s /= (double)N;
    for (int64_t c = 0; c < N; ++c)
        x[c] -= s;
}

static double dot(const double *a, const double *b, int64_t N)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t c = 0; c < N; ++c)
        s += a[c] * b[c];
    return s;
}

/* Solve A p = rhs - mean(rhs) for the mean-zero p.  p holds the initial
 * guess on entry.  Stops when ||b - A p||_2 / ||b||_2 <= tol (true residual),
 * after maxit preconditioned CG iterations, or on stagnation.  Returns 0 on
 * convergence, 1 otherwise; *iters and *relres report what happened. */
static int pcg_solve(const grid_t *g, const double *const beta[3], const double *rhs, double *p,
                     double tol, int maxit, int *iters, double *relres)
{
    int64_t N = cells(g);
    mg_t mg;
    if (mg_build(&mg, g, beta) != 0) {
        mg_free(&mg);
        return -1;
    }
    double *b = (double *)malloc(sizeof(double) * N);
    double *r = (double *)malloc(sizeof(double) * N);
    double *z = (double *)malloc(sizeof(double) * N);
    double *d = (double *)malloc(sizeof(double) * N);
    double *q = (double *)malloc(sizeof(double) * N);
    memcpy(b, rhs, sizeof(double) * N);
    remove_mean(b, N);
    remove_mean(p, N);
    double nb = norm2(b, N);
    if (nb == 0.0) {
        memset(p, 0, sizeof(double) * N);
        *iters = 0;
        *relres = 0.0;
        free(b); free(r); free(z); free(d); free(q);
        mg_free(&mg);
        return 0;
    }
    int it = 0, rc = 1;
    double best = INFINITY;
    int since_best = 0;
    double rel = 0.0;
    /* restarted CG: each restart recomputes the true residual */
    while (it < maxit) {
        apply_A(g, beta, p, q);
        for (int64_t c = 0; c < N; ++c)
            r[c] = b[c] - q[c];
        rel = norm2(r, N) / nb;
        if (rel <= tol) {
            rc = 0;
            break;
        }
        if (rel < 0.5 * best) {
            best = rel;
            since_best = 0;
        } else if (++since_best >= 3) {
            break;   /* stagnated at the rounding floor */
        }
        /* CG on K = -A: K p = -b, residual of that system is -r */
        vcycle(&mg, 0, r, z);  /* z ~ A^-1 r */
        remove_mean(z, N);
        memcpy(d, z, sizeof(double) * N);
        double rz = dot(r, z, N);
        int inner = 0;
        while (it < maxit) {
            apply_A(g, beta, d, q);
            double dq = dot(d, q, N);
            if (dq == 0.0)
                break;
            double alpha = rz / dq;
#pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < N; ++c) {
                p[c] += alpha * d[c];
                r[c] -= alpha * q[c];
            }
            ++it;
            ++inner;
            double rr = norm2(r, N) / nb;
            if (rr <= 0.25 * tol || inner >= 200)
                break;
            vcycle(&mg, 0, r, z);
            remove_mean(z, N);
            double rz2 = dot(r, z, N);
            double bet = rz2 / rz;
            rz = rz2;
#pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < N; ++c)
                d[c] = z[c] + bet * d[c];
        }
    }
    remove_mean(p, N);
    apply_A(g, beta, p, q);
    for (int64_t c = 0; c < N; ++c)
        r[c] = b[c] - q[c];
    rel = norm2(r, N) / nb;
    if (rel <= tol)
        rc = 0;
    *iters = it;
    *relres = rel;
    free(b); free(r); free(z); free(d); free(q);
    mg_free(&mg);
    return rc;
}

EXPORT int ppo_solve(const int64_t *n, const int *bc, double h, const double *bx,
                     const double *by, const double *bz, const double *rhs, double *p,
                     double tol, int maxit, int *iters, double *relres)
{
    grid_t g = make_grid(n, bc, h);
    const double *beta[3] = {bx, by, bz};
    return pcg_solve(&g, beta, rhs, p, tol, maxit, iters, relres);
}

/* Adjoint of p = S(rhs) for L = <g_p, p>: lambda solves A lambda = g_p -
 * mean(g_p) (A is symmetric), g_rhs = lambda, and on every non-wall face
 * g_beta_m[c] = (lambda[c] - lambda[c-e_m]) (p[c] - p[c-e_m]) / h^2; wall
 * faces get 0.  Derivation: A p = b gives dL = lambda^T (db - dA p), and a
 * face coefficient only enters the rows of its two cells. */
EXPORT int ppo_adjoint(const int64_t *n, const int *bc, double h, const double *bx,
                       const double *by, const double *bz, const double *p, const double *gp,
                       double tol, int maxit, double *grhs, double *gbx, double *gby,
                       double *gbz, int *iters, double *relres)
{
    grid_t g = make_grid(n, bc, h);
    const double *beta[3] = {bx, by, bz};
    int64_t N = cells(&g);
    memset(grhs, 0, sizeof(double) * N);
    int rc = pcg_solve(&g, beta, gp, grhs, tol, maxit, iters, relres);
    double *gb[3] = {gbx, gby, gbz};
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(&g, c, ijk);
        for (int m = 0; m < 3; ++m) {
            int64_t dn = neighbour(&g, ijk, m, -1);
            if (dn < 0) {
                gb[m][c] = 0.0;
                continue;
            }
            gb[m][c] = (grhs[c] - grhs[dn]) * (p[c] - p[dn]) / (h * h);
        }
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* General operator: closed links, a diagonal term, excluded cells           */
/* ------------------------------------------------------------------------ */
/*
 * (A_g x)[c] = (A x)[c] - sigma[c] x[c], with the face coefficients of A but
 * interior faces allowed to be 0: a closed link.  Sec. 3.8 blocks the links
 * of a solid by multiplying the link coefficients A1..A6 with the link flags,
 * which is a zero coefficient and a Neumann condition on that face.  The
 * diagonal sigma >= 0 enters in two places of the paper:
 *   - the implicit viscous step (Sec. 3.2.3, eq. muelliptic),
 *     U* - tau mu lap U* = U^n, divided by tau mu_c row by row, is a unit
 *     coefficient Laplacian with sigma_c = 1 / (tau mu_c);
 *   - a Dirichlet branch of the free-surface pressure discretisation
 *     (Sec. 3.7.5, eq. mod_branches): the gradient to an excluded cell is
 *     (p_s - p_c) / delta, so the face adds beta / (h delta) to sigma_c and
 *     -beta p_s / (h delta) to the right-hand side, and its coefficient is 0.
 * A cell with no open face and sigma = 0 is excluded: its row and column
 * vanish and its value is 0.
 */
EXPORT void ppo_apply_gen(const int64_t *n, const int *bc, double h, const double *bx,
                          const double *by, const double *bz, const double *sigma,
                          const double *x, double *y)
{
    grid_t g = make_grid(n, bc, h);
    const double *beta[3] = {bx, by, bz};
    apply_A(&g, beta, x, y);
    if (sigma) {
        int64_t N = cells(&g);
        for (int64_t c = 0; c < N; ++c)
            y[c] -= sigma[c] * x[c];
    }
}

/* diagonal of -A_g: the open face coefficients of the cell / h^2 + sigma */
static void diag_gen(const grid_t *g, const double *const beta[3], const double *sigma,
                     double *dg)
{
    int64_t N = cells(g);
    double ih2 = 1.0 / (g->h * g->h);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        int64_t ijk[3];
        coords(g, c, ijk);
        double s = 0.0;
        for (int m = 0; m < 3; ++m) {
            if (neighbour(g, ijk, m, +1) >= 0)
                s += beta_high(g, beta, ijk, m);
            if (neighbour(g, ijk, m, -1) >= 0)
                s += beta_low(g, beta, ijk, m);
        }
        dg[c] = s * ih2 + (sigma ? sigma[c] : 0.0);
    }
}

/* Solve A_g p = b on the active cells (positive diagonal) by conjugate
 * gradients on -A_g, preconditioned by its diagonal (Jacobi).  When sigma
 * vanishes on every active cell the operator is singular, with the constants
 * on the active set as null space (the caller keeps the active set
 * connected, as the paper's percolation check does): the mean of b over the
 * active cells is removed and p is returned with zero mean there.  Excluded
 * cells get p = 0.  p holds the initial guess on entry.  Returns 0 when
 * ||b - A_g p|| <= tol ||b|| (b masked and, if singular, mean-free), 1
 * otherwise; iters and relres report the iterations and that ratio. */
EXPORT int ppo_solve_gen(const int64_t *n, const int *bc, double h, const double *bx,
                         const double *by, const double *bz, const double *sigma,
                         const double *rhs, double *p, double tol, int maxit, int *iters,
                         double *relres)
{
    grid_t g = make_grid(n, bc, h);
    const double *beta[3] = {bx, by, bz};
    int64_t N = cells(&g);
    double *dg = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N);
    double *s = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    double *d = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
    diag_gen(&g, beta, sigma, dg);
    int singular = 1;
    int64_t nact = 0;
    double bsum = 0.0;
    for (int64_t c = 0; c < N; ++c) {
        if (dg[c] > 0.0) {
            ++nact;
            bsum += rhs[c];
            if (sigma && sigma[c] != 0.0)
                singular = 0;
        }
    }
    double bmean = (singular && nact) ? bsum / (double)nact : 0.0;
    for (int64_t c = 0; c < N; ++c) {
        b[c] = dg[c] > 0.0 ? rhs[c] - bmean : 0.0;
        if (!(dg[c] > 0.0))
            p[c] = 0.0;
    }
    double nb = norm2(b, N);
    int rc = 1, it = 0;
    double rel = 0.0;
    if (nb == 0.0) {
        memset(p, 0, sizeof(double) * N);
        *iters = 0;
        *relres = 0.0;
        free(dg); free(b); free(s); free(z); free(d); free(q);
        return 0;
    }
    /* K = -A_g is positive (semi)definite on the active set: K p = -b.
     * s = -b - K p = -(b - A_g p) is the residual of that system. */
    ppo_apply_gen(n, bc, h, bx, by, bz, sigma, p, q);
    for (int64_t c = 0; c < N; ++c) {
        s[c] = dg[c] > 0.0 ? -(b[c] - q[c]) : 0.0;
        z[c] = dg[c] > 0.0 ? s[c] / dg[c] : 0.0;
        d[c] = z[c];
    }
    double rs = dot(s, z, N);
    while (it < maxit) {
        rel = norm2(s, N) / nb;
        if (rel <= tol)
            break;
        ppo_apply_gen(n, bc, h, bx, by, bz, sigma, d, q);
        for (int64_t c = 0; c < N; ++c)
            q[c] = dg[c] > 0.0 ? -q[c] : 0.0;       /* q = K d */
        double dq = dot(d, q, N);
        if (!(dq > 0.0))
            break;
        double alpha = rs / dq;
        for (int64_t c = 0; c < N; ++c) {
            p[c] += alpha * d[c];
            s[c] -= alpha * q[c];
            z[c] = dg[c] > 0.0 ? s[c] / dg[c] : 0.0;
        }
        double rs2 = dot(s, z, N);
        double bet = rs2 / rs;
        rs = rs2;
        for (int64_t c = 0; c < N; ++c)
            d[c] = z[c] + bet * d[c];
        ++it;
    }
    if (singular && nact) {
        double m = 0.0;
        for (int64_t c = 0; c < N; ++c)
            if (dg[c] > 0.0)
                m += p[c];
        m /= (double)nact;
        for (int64_t c = 0; c < N; ++c)
            if (dg[c] > 0.0)
                p[c] -= m;
    }
    /* true residual */
    ppo_apply_gen(n, bc, h, bx, by, bz, sigma, p, q);
    for (int64_t c = 0; c < N; ++c)
        s[c] = dg[c] > 0.0 ? b[c] - q[c] : 0.0;
    rel = norm2(s, N) / nb;
    rc = rel <= tol ? 0 : 1;
    *iters = it;
    *relres = rel;
    free(dg); free(b); free(s); free(z); free(d); free(q);
    return rc;
}
