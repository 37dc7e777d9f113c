/*
 * pp_kernels.h -- single-kernel entry points of the pressure-projection
 * library, for component tests and kernel timing.
 *
 * These expose the building blocks of the multigrid V-cycle one launch at a
 * time, on caller-provided FP64 device arrays, with the same layout rules as
 * pp.h (cell arrays (nz, ny, nx), low-face beta arrays, walls encoded by the
 * grid's bc).  The V-cycle itself is the in-code geometric multigrid of the
 * paper (Sec. 3.7.3, grids of 2^n cells per direction, user-set numbers of
 * relaxations on the way down and up); its smoother is the red-black
 * Gauss-Seidel of Sec. 3.7.1 (eq. beta_pressure) with over-relaxation 1.
 * Transfer operators are not given in the paper; the readings used:
 *   restriction   r_H = mean of the 8 fine residuals of a coarse cell,
 *   prolongation  cell-centred, per axis between the parent (weight 1 - w)
 *                 and the next coarse cell on the fine cell's side (w), the
 *                 axes composed as a product; w follows the face
 *                 coefficients (pp_k_prolong_weights; 1/4 for equal ones,
 *                 i.e. trilinear interpolation); at a wall the missing coarse
 *                 neighbour is the parent itself,
 *   coarse beta   the mean of two estimates of the conductance between two
 *                 coarse cell centres (pp_k_coarsen_beta).
 * Each call validates its arguments, enqueues on `hip_stream` (NULL = default
 * stream) and returns a pp_status.
 */
#ifndef PP_KERNELS_H
#define PP_KERNELS_H

#include <stdint.h>

#include "pp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* `sweeps` red-black Gauss-Seidel sweeps with over-relaxation on A e = r
 * (Sec. 3.7.1, eq. beta_pressure; one sweep = all red cells (i+j+k even), then
 * all black cells), each cell update
 *   e_c <- (1 - omega) e_c + omega (sum_nb beta_f e_nb - h^2 r_c) / sum_nb beta_f,
 * 0 < omega < 2 (1: plain Gauss-Seidel).  zero_init = 1 treats e as zero on
 * entry (e need not be initialised).  beta_*: fine beta with wall faces
 * already 0 or not (wall entries ignored).  Periodic directions need an even
 * cell count (consistent colouring). */
int pp_k_smooth(const pp_grid *grid, const double *beta_x, const double *beta_y,
                const double *beta_z, const double *r, double *e, int32_t sweeps,
                int32_t zero_init, double omega, void *hip_stream);

/* One fused red-black sweep, out of place: e_out = sweep(e_in), the first
 * colour updated first (first_colour 0: red, (i+j+k) even; 1: black) and the
 * second colour from the new first-colour values.  The same cell update as
 * two colour passes of pp_k_smooth, relaxation omega included (results agree
 * to rounding: the compiler may contract the products into fused
 * multiply-adds differently).  e_in and
 * e_out must not alias; zero_init = 1 treats e_in as zero (it is not read).
 * nx must be even, and so must the cell count of every periodic direction;
 * an x-y plane must stay below 2^31 bytes; all arrays 16-byte aligned (the
 * kernel reads x-pairs of cells as vectors). */
int pp_k_smooth_fused(const pp_grid *grid, const double *beta_x, const double *beta_y,
                      const double *beta_z, const double *r, const double *e_in, double *e_out,
                      int32_t first_colour, int32_t zero_init, double omega, void *hip_stream);

/* Two red-black sweeps in one pass on FP32 arrays (the kernel the FP32 V-cycle
 * uses on large levels): e_out = sweep(sweep(e_in)), each sweep the first
 * colour first as in pp_k_smooth_fused, with relaxation omega (folded into
 * the reciprocal diagonal: e <- (1 - omega) e + (omega / diag) (sum - h^2 r)).
 * Arithmetic is FP32 with the hardware reciprocal of the diagonal (within
 * 1 ulp), so results agree with the FP64 sweeps of the same FP32 inputs to
 * FP32 rounding, not bit for bit.
 * e_in and e_out must not alias; zero_init = 1 treats e_in as zero (it is not
 * read).  Every cell count must be >= 8; nx must be even, and so must the
 * cell count of every periodic direction; an x-y plane must stay below 2^31
 * bytes; all arrays 16-byte aligned. */
int pp_k_smooth2_fused_f32(const pp_grid *grid, const float *beta_x, const float *beta_y,
                           const float *beta_z, const float *r, const float *e_in, float *e_out,
                           int32_t first_colour, int32_t zero_init, double omega,
                           void *hip_stream);

/* pp_k_smooth2_fused_f32 (regular pass: e_in is read) that also forms
 * *dot = sum over all cells of r[c] * e_out[c], with r the pass's own
 * right-hand side: the product (in units of the V-cycle's scale) that the
 * FP32 V-cycle's last fine-level pass hands to the outer conjugate-gradient
 * iteration.  dot: one FP64 device value, 8-byte aligned.  e_out is the same
 * as from pp_k_smooth2_fused_f32, bit for bit; each product r[c] e_out[c] is
 * formed in FP64 from the h^2 r[c] the sweep carries (FP32), the sum in FP64
 * from per-workgroup partials in a fixed order.  Allocates its partial-sum
 * scratch and waits for the stream (a component-test entry). */
int pp_k_smooth2_fused_dot_f32(const pp_grid *grid, const float *beta_x, const float *beta_y,
                               const float *beta_z, const float *r, const float *e_in,
                               float *e_out, int32_t first_colour, double omega, double *dot,
                               void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same pass as
 * pp_k_smooth2_fused_dot_f32, with the same arguments and the same results
 * bit for bit (e_out and *dot), that allocates nothing and does not wait for
 * the stream.  Its workgroup partial sums go to a static device array of
 * 65,536 FP64 values (512 KiB) that each GPU the library runs on holds until
 * the process ends; grids needing more partials than that,
 * ceil(nx/64) * ceil(ny/8) * ceil(nz/8) > 65,536 (512^3 needs 32,768), are
 * rejected with PP_EINVAL.  Every partial the sum reads is written by the
 * same call, so nothing carries over between calls.  All calls on one GPU
 * share the array: calls that overlap in time on one GPU (different streams
 * or threads) race and must be serialised by the caller.  hip_stream must
 * belong to the calling thread's current device (NULL = its default
 * stream).  *dot is ready when the stream reaches the end of the call. */
int pp_k_smooth2_fused_dot_f32_noalloc(const pp_grid *grid, const float *beta_x,
                                       const float *beta_y, const float *beta_z, const float *r,
                                       const float *e_in, float *e_out, int32_t first_colour,
                                       double omega, double *dot, void *hip_stream);

/* rH[C] = (1/8) sum over the 8 fine cells c of C of (r - A e)[c].
 * grid: the fine grid (all n even); rH has n/2 cells per direction; beta,
 * e and r 16-byte aligned. */
int pp_k_resid_restrict(const pp_grid *grid, const double *beta_x, const double *beta_y,
                        const double *beta_z, const double *e, const double *r, double *rH,
                        void *hip_stream);

/* e += P eH, trilinear cell-centred prolongation (3/4 parent, 1/4 the next
 * coarse cell per axis; at a wall the parent itself): the weighted
 * prolongation below with every weight 1/4.  grid: the fine grid (all n
 * even); eH has n/2 cells per direction; e 16-byte aligned. */
int pp_k_prolong_add(const pp_grid *grid, const double *eH, double *e, void *hip_stream);

/* Prolongation weights of every cell of a level (the multigrid V-cycle's
 * interpolation follows the coefficients; the paper gives no transfer
 * operators).  Along an axis a fine cell lies between its parent's centre
 * and the next coarse centre on its side; over that interval the links are
 * half the link between the two children (coefficient gn), the cell's outer
 * face (gm) and half the link beyond it (gf), and the weight of the next
 * coarse cell is the near half link's share of their series resistance:
 *   w = gm gf / (gm gf + gn (2 gf + gm))      (0 when the denominator is 0)
 * i.e. 1/4 for equal coefficients, near 0 for a cell tied to its parent by a
 * strong link and to the next cell through weak ones, 0 at a wall.  For an
 * even index i along the axis gn, gm, gf are the faces i+1, i, i-1, for an
 * odd one i, i+1, i+2 (wrapped; in a wall direction the face of wrapped
 * index 0 counts as 0).  beta_*: FP64 n cells each.  w: n 32-bit words,
 * written: the x, y and z weights as 8-bit fractions q/256 in bits 0-7,
 * 8-15 and 16-23, q = min(255, floor(256 w + 1/2)); bits 24-31 zero. */
int pp_k_prolong_weights(const pp_grid *grid, const double *beta_x, const double *beta_y,
                         const double *beta_z, uint32_t *w, void *hip_stream);

/* e += P eH with the weights of pp_k_prolong_weights (fine-grid cells): per
 * axis (1 - w) times the parent plus w times the next coarse cell on the
 * fine cell's side (the parent itself at a wall), the three axes composed
 * as a product.  grid: the fine grid (all n even); eH has n/2 cells per
 * direction; e 16-byte and w 8-byte aligned. */
int pp_k_prolong_add_weighted(const pp_grid *grid, const double *eH, const uint32_t *w,
                              double *e, void *hip_stream);

/* Coarse face coefficients (wall faces stay 0).  Each of the 4 fine rows
 * that cross a coarse face I contributes its faces lo = 2I-1, mid = 2I and
 * hi = 2I+1 along the normal; the coarse coefficient is the mean of
 *   (a) the mean of the 4 mid faces (the rows in parallel, each taken at the
 *       coarse face: exact when the coefficients vary only across the face)
 *   (b) the mean of the 4 series coefficients 2 / (1/(2 lo) + 1/mid + 1/(2 hi))
 *       (each row's links in series between the two coarse centres: exact
 *       when they vary only along the normal; 0 if a link is closed).
 * (a) overrates a face that cuts through a small inclusion of large
 * coefficient, (b) ignores flow between the rows.  grid: the fine grid;
 * outputs have n/2 cells each. */
int pp_k_coarsen_beta(const pp_grid *grid, const double *beta_x, const double *beta_y,
                      const double *beta_z, double *bH_x, double *bH_y, double *bH_z,
                      void *hip_stream);

/* One V-cycle of the context's hierarchy, in its configured precision, for
 * A e = r (r mean-zero FP64, n cells; e written, FP64). */
int pp_vcycle(pp_ctx *ctx, const double *r, double *e);

/* Plain device copy kernel dst[i] = src[i], i < count (bandwidth reference). */
int pp_k_copy(const double *src, double *dst, int64_t count, void *hip_stream);

/* Kernel timing on the context's stream: every launch of a fine-level kernel
 * whose kind bit is set in `mask` (bit k = 1 << PP_KT_*) carries a pair of
 * HIP events that its dispatch stamps with its own start and end
 * (hipExtLaunchKernel), and its duration is accumulated per kind; mask 0
 * turns timing off.  pp_timing_get reports launches and total ms since the
 * last reset.  Events are read (after waiting for the stream) when queried,
 * reset, turned off, or when the pool of 8192 pairs runs out. */
enum {
    PP_KT_SMOOTH = 0,          /* fine-level red-black half sweep */
    PP_KT_RESTRICT = 1,        /* fine-level residual + restriction */
    PP_KT_PROLONG = 2,         /* fine-level prolongation + correction */
    PP_KT_OUTER_APPLY = 3,     /* FP64 search direction + operator apply (+ dot), outer loop */
    PP_KT_OUTER_UPDATE = 4,    /* FP64 vector update (+ norms) of the outer loop */
    PP_KT_COUNT = 5
};
int pp_timing_enable(pp_ctx *ctx, int32_t mask);
int pp_timing_reset(pp_ctx *ctx);
int pp_timing_get(pp_ctx *ctx, int32_t kind, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* PP_KERNELS_H */
