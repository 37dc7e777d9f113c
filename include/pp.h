/*
 * pp.h -- C ABI of the MI355X (gfx950) pressure-projection library.
 *
 * The library performs the projection step of a one-fluid incompressible
 * Navier-Stokes method on a staggered (MAC) grid (paper Sec. 3.2):
 *
 *   u = u* - dt * beta * G p                                 (eq. fotm)
 *   D (beta G p) = D u* / dt,   so that D u = 0               (eqs. cont-eq1, poisson)
 *
 * with beta = 1/rho on the cell faces (Sec. 3.7.1: the coefficients of the
 * pressure system are interpolations of 1/rho), D the MAC divergence
 * (eq. cont2) and G the face gradient.  Written as the paper's seven-point
 * system (Sec. 3.7.1) the operator has link coefficients A1..A6 = beta_f / h^2
 * and A7 = A1 + ... + A6.  Walls are Neumann boundaries for p: the link
 * coefficient of a wall face is zero (Sec. 3.8) and its normal velocity is 0.
 *
 * ------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ------------------------------------------------------------------------
 *  - Every array argument is a DEVICE pointer (hipMalloc'd or torch CUDA
 *    tensor storage) to contiguous FP64 data owned by the caller.  The
 *    library never frees or retains caller pointers after a call returns.
 *  - Cell arrays have shape (nz, ny, nx) in C order (x fastest).
 *  - A face array for direction m has the same shape; entry c is the LOW
 *    face of cell c in direction m (between c - e_m and c).
 *  - Direction m is periodic (PP_PERIODIC: c - e_m wraps) or walled
 *    (PP_WALL: the entry with c_m == 0 is the wall face; its value is
 *    ignored on input and treated as zero; the upper wall face is implicit).
 *  - Work is enqueued on the HIP stream given to pp_setup, and outputs are
 *    ready in stream order.  Calls that report a convergence result
 *    (pp_solve, pp_solve_adjoint) block the host until that result is known;
 *    the work after it (a solve's gauge, the adjoint's face products) may
 *    still be queued when they return.  Calls that load coefficients wait
 *    for their validity check; the others only enqueue work.
 *  - The operator is singular (constants span its null space): solves remove
 *    the mean of the right-hand side and return the mean-zero solution.
 *  - A context is used by one host thread at a time.
 *
 * Errors: every int-returning function returns PP_OK (0) or a negative
 * pp_status.  Argument validation happens before any GPU work, so PP_EINVAL
 * leaves all outputs untouched.  pp_strerror() names a code; pp_last_error()
 * gives the detail text of the most recent failure on the calling thread.
 */
#ifndef PP_H
#define PP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_ctx pp_ctx;

typedef enum {
    PP_OK = 0,
    PP_EINVAL = -1,      /* bad argument (null pointer, bad size, bad option) */
    PP_ENOMEM = -2,      /* device or host allocation failed */
    PP_EHIP = -3,        /* a HIP runtime call failed */
    PP_ENOCONV = -4,     /* not converged within max_outer: p holds the best iterate */
    PP_EDIVERGED = -5    /* NaN/Inf or residual blow-up: p is undefined */
} pp_status;

enum { PP_PERIODIC = 0, PP_WALL = 1 };

/* arithmetic of the multigrid preconditioner; the outer loop, its residual,
 * the coarsest-grid solve and the projection are always FP64 */
enum { PP_FP64 = 0, PP_MIXED_FP32 = 1, PP_MIXED_FP16 = 2 };

/* outer iteration around the V-cycle */
enum { PP_OUTER_PCG = 0, PP_OUTER_DC = 1 };
/* multigrid cycle: how often each level takes its coarse correction */
enum { PP_CYCLE_V = 0, PP_CYCLE_W = 1, PP_CYCLE_F = 2 };

typedef struct {
    int32_t n[3];        /* cells per direction {nx, ny, nz}; see pp_setup */
    double h;            /* cell edge (cubic cells) */
    int32_t bc[3];       /* PP_PERIODIC or PP_WALL per direction {x, y, z} */
} pp_grid;

typedef struct {
    int32_t precision;   /* PP_FP64 / PP_MIXED_FP32 / PP_MIXED_FP16 */
    int32_t outer;       /* PP_OUTER_PCG (flexible CG) or PP_OUTER_DC (defect correction) */
    int32_t nu_pre;      /* red-black Gauss-Seidel sweeps before coarsening (>= 1) */
    int32_t nu_post;     /* sweeps after the coarse correction (>= 1) */
    int32_t max_outer;   /* outer iterations before PP_ENOCONV (1..4096) */
    int32_t warm_start;  /* 1: pp_solve starts from the p passed in; 0: from p = 0 */
    int32_t fallback;    /* 1: on stagnation of a mixed solve, continue with FP64 V-cycles */
    int32_t coarse_graph; /* 1: replay the coarse levels of each V-cycle from a HIP graph
                            captured in pp_setup (same kernels, same order, same results);
                            0 (default): launch them one by one, which measured faster since
                            the iterations are queued ahead of the GPU */
    int32_t nu_coarse;   /* red-black sweeps before and after the coarse correction on the
                            smallest levels (at most 4096 cells each), which run inside one
                            workgroup; they are cheap there and set the outer iteration
                            count at high density ratios (1..16) */
    double omega;        /* over-relaxation of the red-black smoother on every level
                            (Sec. 3.7.1, eq. beta_pressure: p <- (1 - omega) p + omega p_GS),
                            in (0, 2); the same factor before and after the coarse
                            correction keeps the V-cycle symmetric */
    int32_t cycle;       /* PP_CYCLE_V (default): each level's coarse correction once (the
                            paper's V-cycle, Sec. 3.7.3).  PP_CYCLE_W: twice on every level
                            above the single-workgroup tail, the second pass starting from
                            the first one's correction (a W-cycle; symmetric like the V-cycle).
                            PP_CYCLE_F: the first pass an F-cycle, the second a V-cycle (level
                            k is visited k + 1 times, not 2^k; not symmetric, so meant for the
                            flexible PCG).  W and F take fewer outer iterations where isolated
                            gas bubbles defeat the coarse grids (20 bubbles at density ratio
                            1000, 128^3: 23 -> 11 for W), at more coarse-level latency per
                            iteration; other values: PP_EINVAL */
    int32_t coarsest;    /* the hierarchy stops halving at a level of at most this many
                            cells, 1..1024 (default 64: 4^3 for power-of-two grids); that
                            level is solved with an FP64 pseudo-inverse (Sec. 3.7.3, the
                            coarsest-grid solve), held in LDS up to 64 cells */
} pp_opts;

#define PP_HIST 128

typedef struct {
    int32_t outer_iters; /* outer iterations done */
    int32_t vcycles;     /* V-cycles applied */
    int32_t fell_back;   /* 1 if a mixed solve switched to FP64 V-cycles */
    int32_t status;      /* the pp_status the call returned */
    double rel_res;      /* final ||b - A p||_2 / ||b||_2 (b mean-removed) */
    double res_hist[PP_HIST]; /* relative residual after each outer iteration */
    double ms;           /* host wall time of the call, milliseconds */
} pp_stats;

/* Fill *o with the defaults: mixed FP32, PCG, nu_pre = nu_post = 2,
 * max_outer = 500, warm_start = 0, fallback = 1, coarse_graph = 0, nu_coarse = 4,
 * omega = 1.2, cycle = PP_CYCLE_V, coarsest = 64. */
void pp_opts_default(pp_opts *o);

/* Face coefficients from cell densities, beta_m[c] = 2 / (rho[c - e_m] + rho[c])
 * (arithmetic averaging of rho on the two cells of a face; Sec. 3.7.1 builds
 * the coefficients from 1/rho interpolated to the faces).  Wall faces get 0.
 * rho: n cells, all > 0.  beta_x/y/z: n cells each, written.  Needs no
 * context; work goes on `hip_stream` (NULL = default stream). */
int pp_face_coeffs(const pp_grid *grid, const double *rho, double *beta_x, double *beta_y,
                   double *beta_z, void *hip_stream);

/* Build a solver context for one set of face coefficients beta = 1/rho_f
 * (the pressure operator of eq. poisson and its multigrid hierarchy, Sec. 3.7.3).
 * Grid: every n[m] >= 4; the grid is halved in all directions while all
 * n[m] are even and >= 8 and the level has more than opts.coarsest cells; the
 * coarsest level reached must have at most 1024 cells (every power-of-two
 * grid qualifies).  h > 0.  beta_x/y/z: n cells
 * each, finite; every non-wall face must have beta > 0 (a connected domain).
 * The context copies beta (caller may free it afterwards), builds the
 * multigrid hierarchy and the FP64 pseudo-inverse of the coarsest operator,
 * and owns all device scratch; later calls allocate nothing.  opts may be
 * NULL (defaults).  hip_stream: the hipStream_t to use (NULL = default).
 * On success *out receives the context; release it with pp_destroy. */
int pp_setup(const pp_grid *grid, const double *beta_x, const double *beta_y,
             const double *beta_z, const pp_opts *opts, void *hip_stream, pp_ctx **out);

/* General operator (Sec. 3.8 solid link flags; Sec. 3.2.3 implicit viscous
 * step; Sec. 3.7.5 free-surface Dirichlet branches):
 *
 *   (A_g x)_c = sum_m [beta_m(c+e_m)(x_{c+e_m} - x_c) - beta_m(c)(x_c - x_{c-e_m})] / h^2
 *               - sigma_c x_c
 *
 * Differences from pp_setup:
 *  - beta may be 0 on interior faces: a closed link (the paper's link flags
 *    zero A1..A6 across a solid), a Neumann condition on that face.  Every
 *    non-wall face must be a finite non-negative number.
 *  - sigma (n cells, finite, >= 0) is a diagonal term; NULL means none.  The
 *    implicit viscous step U* - tau mu lap U* = U^n, divided by tau mu_c row
 *    by row, is this operator with beta = 1, sigma_c = 1/(tau mu_c) and
 *    rhs = -U^n / (tau mu_c).  A free-surface Dirichlet branch (gradient
 *    (p_s - p_c)/delta to the interface) is a closed link plus
 *    sigma_c += beta/(h delta) and rhs_c -= beta p_s/(h delta).
 *  - a cell with no open face and sigma = 0 is excluded: pp_solve returns 0
 *    there and ignores its right-hand side.
 *  - with no positive sigma the operator is singular, with the constants on
 *    the active cells as null space: pp_solve removes the mean of the rhs
 *    over the active cells and returns p with zero mean over them.  The
 *    active cells must then be connected (the caller checks this, as the
 *    paper leaves it to a separate percolation check); otherwise the solve
 *    stalls and returns PP_ENOCONV.  With a positive sigma nothing is removed.
 * On a context made here every later call uses A_g: pp_apply returns A_g x;
 * pp_divergence gives closed links no flux; pp_project writes u = 0 on
 * closed links (as on walls); pp_solve_adjoint writes g_beta = 0 on closed
 * links, and dL/d sigma_c = g_rhs_c * p_c follows from its outputs.
 * Returns as pp_setup; PP_EINVAL also when no cell is active. */
int pp_setup_general(const pp_grid *grid, const double *beta_x, const double *beta_y,
                     const double *beta_z, const double *sigma, const pp_opts *opts,
                     void *hip_stream, pp_ctx **out);

/* New coefficients from the cell densities (Sec. 3.2: beta = 1/rho at the
 * faces, the interpolation of pp_face_coeffs): beta = 2 / (rho_L + rho_R) on
 * every non-wall face, computed on the device together with the hierarchy
 * rebuild of pp_update_coeffs, so the coefficients are the ones
 * pp_face_coeffs followed by pp_update_coeffs would load, bit for bit, in one
 * pass over memory.  rho: device (nz, ny, nx) FP64 array, read only, owned by
 * the caller (16-byte alignment selects the one-pass kernel).  For contexts
 * made by pp_setup only.  PP_EINVAL if a cell's density or a resulting face
 * coefficient is not a finite positive number; the context's coefficients
 * are then undefined until a later successful update.  The context keeps its
 * own copy of rho (N doubles, allocated by the first call; the caller may
 * overwrite rho afterwards): until the next coefficient update, pp_solve's
 * search-direction pass and pp_project form beta from it with the same
 * expression (same bits) instead of reading the three coefficient arrays. */
int pp_update_density(pp_ctx *ctx, const double *rho);

/* New coefficients for a context made by pp_setup_general (same grid);
 * sigma must be NULL exactly when it was NULL at setup.  As pp_update_coeffs
 * otherwise. */
int pp_update_general(pp_ctx *ctx, const double *beta_x, const double *beta_y,
                      const double *beta_z, const double *sigma);

/* Replace the face coefficients of an existing context (same grid), rebuilding
 * the hierarchy in place without reallocating.  Same rules as pp_setup (as
 * pp_update_general with sigma NULL for a general context without sigma).  If
 * the coefficients are rejected (PP_EINVAL: a non-wall face that is not a
 * finite positive number), the context's coefficients are undefined until a
 * later successful update. */
int pp_update_coeffs(pp_ctx *ctx, const double *beta_x, const double *beta_y,
                     const double *beta_z);

/* out = scale * D u with D the MAC divergence (eq. cont2); wall faces count
 * as zero flux whatever their stored value.  u_x/u_y/u_z, out: n cells.
 * The pressure right-hand side of eq. poisson is scale = 1/dt. */
int pp_divergence(pp_ctx *ctx, const double *u_x, const double *u_y, const double *u_z,
                  double scale, double *out);

/* out = A x, the FP64 pressure operator of eq. poisson, D(beta G x) (x, out: n
 * cells; must not alias). */
int pp_apply(pp_ctx *ctx, const double *x, double *out);

/* The pressure solve of eq. poisson (Sec. 3.7: multigrid, Sec. 3.7.3, as the
 * preconditioner of conjugate gradients or of defect correction).
 * Solve A p = rhs - mean(rhs) to ||b - A p||_2 <= tol ||b||_2 (b = rhs -
 * mean(rhs)) and return the mean-zero p.  rhs, p: n cells; p is read as the
 * initial guess when opts.warm_start is set, and written.  tol in (0, 1).
 * stats may be NULL.  Returns PP_OK, PP_ENOCONV (p = best iterate, stats
 * filled) or PP_EDIVERGED (p undefined). */
int pp_solve(pp_ctx *ctx, const double *rhs, double *p, double tol, pp_stats *stats);

/* Projection (eq. fotm): u_m = us_m - dt * beta_m * (p[c] - p[c - e_m]) / h on
 * every non-wall face, u_m = 0 on wall faces.  us_x/y/z, p, u_x/y/z: n cells.
 * u may alias us (in-place update); p must not alias u. */
int pp_project(pp_ctx *ctx, const double *us_x, const double *us_y, const double *us_z,
               const double *p, double dt, double *u_x, double *u_y, double *u_z);

/* One whole projection step of the fractional-step method (Sec. 3: the
 * density-weighted pressure equation, eq. poisson, and the velocity update,
 * eq. fotm), in one call: pp_update_density(rho), rhs = pp_divergence(us,
 * 1/dt), pp_solve(rhs, p, tol, stats) and pp_project(us, p, dt, u), with the
 * same kernels in the same order and so the same results, bit for bit.  The
 * host waits only where the solve needs its results: the density check is
 * read back with the solve's initial residual instead of on its own, and the
 * projection is queued before the host waits for the confirming final
 * residual (queued again should the iteration go on; after that wait when a
 * u_m aliases us_m, as a projection in place cannot be redone).  For contexts
 * made by pp_setup.
 * rho, us_x/y/z: read only; rhs (scratch that receives D us / dt), p (initial
 * guess when opts.warm_start is set) and u_x/y/z: written; all n cells, owned
 * by the caller.  u_m may alias us_m; no other two arrays may alias.  dt
 * finite and nonzero, tol in (0, 1); stats as pp_solve's (may be NULL).
 * Returns PP_OK; PP_ENOCONV (p the best iterate, u projected with it);
 * PP_EINVAL for bad arguments (nothing done) or a rejected density (as
 * pp_update_density: the coefficients are then undefined until a later
 * successful update, and rhs, p and u are undefined); PP_EDIVERGED. */
int pp_step(pp_ctx *ctx, const double *rho, const double *us_x, const double *us_y,
            const double *us_z, double dt, double tol, double *rhs, double *p, double *u_x,
            double *u_y, double *u_z, pp_stats *stats);

/* Adjoint of the pressure solve of eq. poisson, derived from A's symmetry
 * (the paper gives no adjoint): for p = pp_solve(rhs) and a loss L with
 * dL/dp = g_p, solves
 * A lambda = g_p - mean(g_p) with the same hierarchy (A is symmetric) and
 * writes g_rhs = lambda (mean zero) and, on every non-wall face,
 * g_beta_m[c] = (lambda[c] - lambda[c - e_m]) (p[c] - p[c - e_m]) / h^2
 * (wall faces 0).  p is the forward solution.  All arrays n cells; tol as in
 * pp_solve; stats may be NULL. */
int pp_solve_adjoint(pp_ctx *ctx, const double *p, const double *g_p, double tol,
                     double *g_rhs, double *g_beta_x, double *g_beta_y, double *g_beta_z,
                     pp_stats *stats);

/* Number of multigrid levels and the dimensions of level `level` (0 = fine). */
int pp_levels(const pp_ctx *ctx, int32_t *nlevels);
int pp_level_dims(const pp_ctx *ctx, int32_t level, int32_t dims[3]);

/* Device bytes held by the context. */
int pp_memory(const pp_ctx *ctx, int64_t *bytes);

void pp_destroy(pp_ctx *ctx);
const char *pp_strerror(int status);
const char *pp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PP_H */
