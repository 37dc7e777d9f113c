// pp_internal.h -- internal declarations shared by the HIP sources of the
// pressure-projection library (kernels + host driver).  Not part of the ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pp {

// Kernel timing without markers: the host driver's timer scope leaves a pair
// of events here, and the next launch made through PP_LAUNCH on the same
// thread hands them to the dispatch itself (hipExtLaunchKernel), so they take
// the kernel's own start and end and no event packet sits between kernels.
struct LaunchTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchTimer g_launch_timer;

#define PP_LAUNCH(kern, grid, block, shmem, stream, ...)                                       \
    do {                                                                                       \
        if (::pp::g_launch_timer.start) {                                                      \
            const ::pp::LaunchTimer pp_lt_ = ::pp::g_launch_timer;                             \
            ::pp::g_launch_timer = ::pp::LaunchTimer{};                                        \
            hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, pp_lt_.start, pp_lt_.stop, \
                                  0, __VA_ARGS__);                                             \
        } else {                                                                               \
            hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);                 \
        }                                                                                      \
    } while (0)

// Cell kernels run 64 x 4 thread blocks (four 64-wide waves, one x-row
// segment per wave), with the z index taken from blockIdx.z.
constexpr int BX = 64;
constexpr int BY = 4;
constexpr int BLOCK = BX * BY;

struct Dims {
    int nx, ny, nz;
};

// 1 = wall in that direction, 0 = periodic.
struct Bc {
    int x, y, z;
};

__host__ __device__ inline size_t cells(Dims d) { return (size_t)d.nx * d.ny * d.nz; }

// levels handled by the single-workgroup tail of the V-cycle
constexpr int TAIL_MAX = 8;
constexpr size_t TAIL_CELLS = 4096;       // a level joins the tail at or below this size
constexpr size_t FUSED_MIN_CELLS = (size_t)1 << 18;   // fused sweeps above 64^3 cells
// FP32 / FP16 storage, whose fused pass does two sweeps per launch, from 32^3 cells
constexpr size_t FUSED2_MIN_CELLS = (size_t)1 << 14;
template <typename T>
constexpr size_t fused_min_cells()
{
    return sizeof(T) == 8 ? FUSED_MIN_CELLS : FUSED2_MIN_CELLS;
}

// The fused sweep addresses a plane through 32-bit byte offsets with one
// reserved out-of-range value: planes must stay below 2^31 bytes.
inline bool fused_plane_fits(Dims d, size_t word)
{
    return (size_t)d.nx * d.ny * word < ((size_t)1 << 31);
}

inline dim3 cell_grid(Dims d)
{
    return dim3((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz);
}

// grid for kernels that give each thread one cell of one colour
inline dim3 colour_grid(Dims d)
{
    int half = (d.nx + 1) / 2;
    return dim3((half + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz);
}

inline size_t grid_blocks(dim3 g) { return (size_t)g.x * g.y * g.z; }

// kernels that also reduce walk RZ planes per block: fewer partial sums
constexpr int RZ = 8;
inline dim3 red_grid(Dims d)
{
    return dim3((d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, (d.nz + RZ - 1) / RZ);
}

// ---------------------------------------------------------------------------
// scalar slots of the device scalar array used by the outer iterations
// ---------------------------------------------------------------------------
enum Slot {
    S_MEAN = 0,     // mean of the right-hand side
    S_RR = 1,       // ||r||^2
    S_BB = 2,       // ||b||^2 (b mean-removed)
    S_RZ = 3,       // r . z (current)
    S_RZOLD = 4,    // r_new . z_old (flexible CG)
    S_ALPHA = 5,
    S_BETA = 6,
    S_USED = 7,     // scale of the right-hand side the V-cycle currently holds
    S_NEXT = 8,     // RMS of the latest residual (scale for the next V-cycle)
    S_XMEAN = 9,    // mean of the iterate (gauge)
    S_COUNT = 10,   // generic count (validation)
    S_DQ = 11,
    S_SBAD = 12,    // sigma entries that are not finite non-negative (validation)
    S_SPOS = 13,    // positive sigma entries
    S_NACT = 14,    // active cells of the general operator
    S_DS = 15,      // V-cycle scale of the latest direction (outer CG)
    S_APREV = 16,   // the previous outer iteration's ALPHA
    S_NSLOTS = 17
};

enum FinalizeOp {
    OP_STORE = 0,   // scal[slot] = sum0
    OP_MEAN = 1,    // scal[slot] = sum0 / N
    OP_INIT = 2,    // RR, BB, S_USED = S_NEXT = rms(r)
    OP_RZ = 3,      // RZ, BETA (flexible Polak-Ribiere)
    OP_ALPHA = 4,   // ALPHA = RZ / DQ
    OP_UPDATE = 5,  // RR, RZOLD, rotate scales
    OP_DC = 6,      // RR, rotate scales
    OP_RZ_T = 7     // as OP_RZ, the partials formed with the V-cycle's scaled right-hand side
};

// ---------------------------------------------------------------------------
// launchers (pp_kernels.hip); T is the storage type of V-cycle data.  `sg` is
// the diagonal term of the general operator A - diag(sigma) on that level,
// stored as h^2 sigma (the unit of the face coefficients in the smoother), or
// null for the pressure operator; cells with no open face and no diagonal
// term are excluded (their correction stays 0).  `omega` is the smoother's
// over-relaxation (eq. beta_pressure): e <- (1 - omega) e + omega e_GS.
// ---------------------------------------------------------------------------
// one colour of a red-black sweep, in place; zero: e is 0 on entry (neither
// the cell nor its neighbours are read); self_zero: the cell's own old value
// is 0 (the second colour of a sweep from zero), its neighbours are read
template <typename T>
void launch_rbgs(Dims d, Bc bc, const T *bx, const T *by, const T *bz, const T *r, T *e,
                 const T *sg, double h2, double omega, int colour, bool zero, bool self_zero,
                 hipStream_t s);
// query (once) the occupancy figures the fused sweep's launch geometry uses;
// called before stream capture so that capture records kernel launches only
template <typename T>
void prepare_fused();
// one fused red-black sweep, e_in -> e_out (must not alias); first_colour 0
// updates red ((i+j+k) even) first, 1 black first; zero: e_in treated as 0
template <typename T>
void launch_rbgs_fused(Dims d, Bc bc, const T *bx, const T *by, const T *bz, const T *r,
                       const T *ein, T *eout, const T *sg, double h2, double omega,
                       int first_colour, bool zero, hipStream_t s);
// Two sweeps in one pass (FP32 and FP16 storage only), out of place, ein and
// eout distinct; needs nz >= 8 (the chunks read four planes beyond their ends).
template <typename T>
void prepare_fused2();
// With part given, an FP32 regular pass without sigma also writes the partial
// sums of r . e_out (its own right-hand side against its output, products in
// FP64), one per workgroup, and returns their number; otherwise returns 0.
template <typename T>
int launch_rbgs_fused2(Dims d, Bc bc, const T *bx, const T *by, const T *bz, const T *r,
                       const T *ein, T *eout, const T *sg, double h2, double omega,
                       int first_colour, bool zero, hipStream_t s, double *part = nullptr);
inline bool fused2_fits(Dims d) { return d.nz >= 8 && d.nx >= 8 && d.ny >= 8; }
template <typename T>
void launch_resid_restrict(Dims fd, Bc bc, const T *bx, const T *by, const T *bz, const T *e,
                           const T *r, const T *sg, T *rH, double ih2, hipStream_t s);
// e += P eH with the prolongation weights w of the fine level (one 32-bit
// word per fine cell: the x, y and z weights as 8-bit fractions of 256 in
// bits 0-7, 8-15, 16-23; null: 1/4 everywhere, trilinear)
template <typename T>
void launch_prolong(Dims fd, Bc bc, const T *eH, T *e, const unsigned *w, hipStream_t s);
// the prolongation weights of a level from its FP64 face coefficients
void launch_prolong_weights(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                            unsigned *w, hipStream_t s);
template <typename T>
void launch_coarsest(int n, const double *pinv, const T *r, T *e, hipStream_t s);
// the V-cycle on nlev levels (the last one the coarsest) in one workgroup;
// input r[0], output e[0] (in place; every level's e is overwritten); warm:
// e[0] holds a correction on entry, which the first level's sweeps start from
template <typename T>
void launch_tail(int nlev, const Dims *d, const double *h2, const void *const (*b)[3], void *const *e,
                 void *const *r, const void *const *sg, const unsigned *const *w, Bc bc,
                 int nu_pre, int nu_post, double omega, const double *pinv, int ncoarse,
                 bool warm, hipStream_t s);
template <typename T>
void launch_convert(size_t n, const double *src, T *dst, hipStream_t s);
template <typename T>
void launch_to_double(size_t n, const T *src, double *dst, hipStream_t s);
// dst = scale * src in the storage type; partials (one per block, at most
// max_blocks, count returned) of the entries whose magnitude is not below `limit`
template <typename T>
int launch_convert_scaled(size_t n, const double *src, double scale, double limit, T *dst,
                          double *part, int max_blocks, hipStream_t s);

void launch_coarsen_beta(Dims fd, Bc bc, const double *bx, const double *by, const double *bz,
                         double *hx, double *hy, double *hz, hipStream_t s);
// one pass: copy + wall zeroing + validity count (partials) + storage copy
// (dstT[0] may be null) + first coarse level; the fine grid's n must all be
// even; returns the number of partial sums written (part null: no count, 0);
// coarseT (may be null): the first coarse level's storage copy too
template <typename T>
int launch_load_coeffs(Dims fd, Bc bc, const double *const src[3], double *const dst[3],
                       T *const dstT[3], double *const coarse[3], unsigned *w0, double *part,
                       hipStream_t s, T *const coarseT[3] = nullptr);
// as launch_load_coeffs with beta computed from the cell densities (the
// arithmetic of launch_face_coeffs), also copying the densities to rcopy; the
// partials also count cells whose density is not a finite positive number
template <typename T>
int launch_load_density(Dims fd, Bc bc, const double *rho, double *const dst[3], T *const dstT[3],
                        double *const coarse[3], double *rcopy, unsigned *w0, double *part,
                        hipStream_t s);
void launch_check_rho(Dims d, const double *rho, double *part, hipStream_t s);
void launch_zero_walls(Dims d, Bc bc, double *bx, double *by, double *bz, hipStream_t s);
// partials of the count of non-wall faces that are not finite positive
// numbers (finite non-negative with allow_zero: closed links allowed)
void launch_check_beta(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                       bool allow_zero, double *part, hipStream_t s);
// partials: [0] sigma entries that are not finite non-negative, [pstride +]
// positive entries
void launch_check_sigma(Dims d, const double *sg, double *part, size_t pstride, hipStream_t s);
// act = cells with an open face or sigma > 0; partials of their count
void launch_active(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                   const double *sg, unsigned char *act, double *part, hipStream_t s);
void launch_coarsen_sigma(Dims fd, const double *sg, double *sH, hipStream_t s);
void launch_mask(size_t n, double *x, const unsigned char *act, hipStream_t s);
void launch_face_coeffs(Dims d, Bc bc, const double *rho, double *bx, double *by, double *bz,
                        hipStream_t s);
// bx/by/bz may be null; when given, closed links (beta = 0) carry no flux
// the divergence of the pressure operator (no face coefficients) with the
// partial sums of out in k_sum's blocks and order; returns their count
int launch_divergence_sum(Dims d, Bc bc, const double *ux, const double *uy, const double *uz,
                          double scale_over_h, double *out, double *part, hipStream_t s);
void launch_divergence(Dims d, Bc bc, const double *ux, const double *uy, const double *uz,
                       double scale_over_h, const double *bx, const double *by, const double *bz,
                       double *out, hipStream_t s);
void launch_apply(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                  const double *x, const double *sg, double *y, double ih2, hipStream_t s);
// rho non-null: beta from the cell densities (as for launch_dir_apply)
void launch_project(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                    const double *rho, const double *usx, const double *usy, const double *usz,
                    const double *p, double dt_over_h, double *ux, double *uy, double *uz,
                    hipStream_t s);
void launch_adjoint_faces(Dims d, Bc bc, const double *lam, const double *p, double ih2,
                          const double *bx, const double *by, const double *bz, double *gx,
                          double *gy, double *gz, hipStream_t s);
void launch_copy(const double *src, double *dst, size_t n, hipStream_t s);
void launch_fill(double *x, size_t n, double v, hipStream_t s);

// reductions and outer-loop kernels (FP64); `part` holds one partial sum per
// block and quantity, quantity q at part[q * pstride + block]
// act may be null (every cell); otherwise only active cells are summed
void launch_sum(Dims d, const double *x, const unsigned char *act, double *part, hipStream_t s);
// narr (at most 4) arrays of n doubles each, one after the other, to pinned,
// coherent host memory, in one kernel
void launch_publish_arrays(const double *const *src, int narr, int n, double *host, hipStream_t s);
// n doubles to pinned, coherent host memory, written by a kernel; a nonzero
// ticket is then written to host[n] (which must exist), after the values
void launch_publish(const double *src, double *host, int n, hipStream_t s, double ticket = 0.0);
// host (optional): pinned, coherent host memory that receives a copy of all
// S_NSLOTS scalars when the operation is done, then the ticket in
// host[S_NSLOTS]
void launch_finalize(const double *part, size_t pstride, int nparts, int op, int slot,
                     double ncells, int first, double *scal, hipStream_t s,
                     double *host = nullptr, double ticket = 0.0);
// returns the number of partial sums written (at most grid_blocks(red_grid(d)))
// whether launch_residual (x given) forms the link coefficients from rho
// rather than reading bx, by, bz: the 2 x 2 kernel on even grids with 16-byte
// aligned arrays
inline bool residual_from_rho(Dims d, const double *rho, const double *b, const double *x,
                              const double *r64)
{
    return rho && d.nx % 2 == 0 && d.ny % 2 == 0 &&
           (((uintptr_t)x | (uintptr_t)b | (uintptr_t)r64 | (uintptr_t)rho) & 15) == 0;
}
int launch_residual(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                    const double *rho, const double *b, const double *scal, double *x, bool zero_x,
                    const double *sg, const unsigned char *act, double *r64, double ih2,
                    double *part, size_t pstride, hipStream_t s);
template <typename T>
void launch_residual_T(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                       const double *b, const double *scal, const double *x, const double *sg,
                       const unsigned char *act, T *rT, double ih2, double *part, hipStream_t s);
template <typename T>
void launch_scale_T(size_t n, const double *r, T *rT, const double *scal, hipStream_t s);
template <typename T>
void launch_axpy_T(size_t n, const T *e, double *x, const double *scal, hipStream_t s);
template <typename T>
void launch_dot_rz(Dims d, const double *r, const T *z, double *part, hipStream_t s);
// Storage of the outer search direction (in units of the V-cycle's scale):
// FP64 with the FP64 preconditioner, FP32 with the mixed ones, whose
// preconditioned residual is itself no more accurate than FP32.  The
// direction only has to agree with its image q, which is formed from the
// stored values.
template <typename T>
struct DirT {
    using type = float;
};
template <>
struct DirT<double> {
    using type = double;
};
// returns the number of partial sums written (at most grid_blocks(red_grid(d)))
// rho non-null: the link coefficients are formed from the cell densities
// (the plain operator whose coefficients came from them), not read from bx..bz.
// The iterate's update (mode): DIR_FIRST none (first iteration: no D_old),
// DIR_HOLD none (its direction waits a pass), DIR_TWO x += APREV * (dnew as
// it was, D_{k-2}) + ALPHA * D_old, the two pending directions.
enum DirMode { DIR_FIRST = 0, DIR_HOLD = 1, DIR_TWO = 2 };
template <typename T>
int launch_dir_apply(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                     const double *rho, const T *z, const typename DirT<T>::type *dold,
                     typename DirT<T>::type *dnew, double *q, double *x, const double *sg,
                     const double *scal, int mode, double ih2, double *part, size_t pstride,
                     hipStream_t s);
template <typename T>
void launch_pcg_update(Dims d, const double *q, double *r, T *rT, const double *scal, double *part,
                       hipStream_t s);
// x += scal[S_ALPHA] * dv, after x += scal[S_APREV] * dv_prev when dv_prev
// is given (the two directions still pending after the last iteration)
template <typename D>
void launch_axpy_dir(size_t n, const D *dv, const D *dv_prev, double *x, const double *scal,
                     hipStream_t s);
// x -= scal[slot] (slot < 0: nothing); with act, excluded cells are set to 0
void launch_sub_mean(size_t n, double *x, const double *scal, int slot, const unsigned char *act,
                     hipStream_t s);

}  // namespace pp
