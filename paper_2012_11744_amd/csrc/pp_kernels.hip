// pp_kernels.hip -- HIP kernels (gfx950) of the pressure-projection library.
//
// Discretisation (paper Sec. 3.1, Sec. 3.7.1): cell-centred p on a MAC grid
// with cubic cells of edge h; face coefficient beta = 1/rho; the operator
//   (A x)_c = sum_m [ beta_m(c+e_m) (x_{c+e_m} - x_c) - beta_m(c) (x_c - x_{c-e_m}) ] / h^2
// is the seven-point system of Sec. 3.7.1 (A1..A6 = beta/h^2, A7 = their sum).
// Walls (Sec. 3.8) zero the link coefficient of the wall face.  Every kernel
// masks wall links explicitly from the grid's bc, so stored wall entries are
// never used; periodic neighbours wrap.
//
// The kernels are memory-bound stencils: one thread per cell (or per cell of
// one colour), 64-wide rows in x so each wave reads contiguous x segments,
// neighbours in y and z served by L2.  Reductions are two-stage and fixed
// order (wave shuffle -> LDS -> one partial per block -> one finalising
// block), so every result is bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "pp_device.h"
#include "pp_internal.h"

namespace pp {

thread_local LaunchTimer g_launch_timer;

template <typename T>
__device__ __forceinline__ typename Acc<T>::type ld(const T *p, size_t i)
{
    return static_cast<typename Acc<T>::type>(p[i]);
}

struct Nb {
    size_t c, xm, xp, ym, yp, zm, zp;
    bool wxl, wxh, wyl, wyh, wzl, wzh;   // link crosses a wall
};

__device__ __forceinline__ Nb neighbours(Dims d, Bc bc, int i, int j, int k)
{
    const size_t sy = (size_t)d.nx;
    const size_t sz = (size_t)d.nx * d.ny;
    Nb n;
    n.c = (size_t)k * sz + (size_t)j * sy + (size_t)i;
    const size_t row = n.c - (size_t)i;
    n.xm = row + (size_t)(i == 0 ? d.nx - 1 : i - 1);
    n.xp = row + (size_t)(i == d.nx - 1 ? 0 : i + 1);
    const size_t col = n.c - (size_t)j * sy;
    n.ym = col + (size_t)(j == 0 ? d.ny - 1 : j - 1) * sy;
    n.yp = col + (size_t)(j == d.ny - 1 ? 0 : j + 1) * sy;
    const size_t pil = n.c - (size_t)k * sz;
    n.zm = pil + (size_t)(k == 0 ? d.nz - 1 : k - 1) * sz;
    n.zp = pil + (size_t)(k == d.nz - 1 ? 0 : k + 1) * sz;
    n.wxl = bc.x && i == 0;
    n.wxh = bc.x && i == d.nx - 1;
    n.wyl = bc.y && j == 0;
    n.wyh = bc.y && j == d.ny - 1;
    n.wzl = bc.z && k == 0;
    n.wzh = bc.z && k == d.nz - 1;
    return n;
}

// the six link coefficients of a cell (0 across walls)
template <typename T>
struct Links {
    typename Acc<T>::type xl, xh, yl, yh, zl, zh;
};

template <typename T>
__device__ __forceinline__ Links<T> links(const Nb &n, const T *bx, const T *by, const T *bz)
{
    using C = typename Acc<T>::type;
    Links<T> L;
    L.xl = n.wxl ? C(0) : ld(bx, n.c);
    L.xh = n.wxh ? C(0) : ld(bx, n.xp);
    L.yl = n.wyl ? C(0) : ld(by, n.c);
    L.yh = n.wyh ? C(0) : ld(by, n.yp);
    L.zl = n.wzl ? C(0) : ld(bz, n.c);
    L.zh = n.wzh ? C(0) : ld(bz, n.zp);
    return L;
}

// h^2 (A x)_c
template <typename T, typename X>
__device__ __forceinline__ typename Acc<T>::type flux_sum(const Nb &n, const Links<T> &L, const X *x)
{
    using C = typename Acc<T>::type;
    const C xc = static_cast<C>(x[n.c]);
    return L.xh * (static_cast<C>(x[n.xp]) - xc) - L.xl * (xc - static_cast<C>(x[n.xm])) +
           L.yh * (static_cast<C>(x[n.yp]) - xc) - L.yl * (xc - static_cast<C>(x[n.ym])) +
           L.zh * (static_cast<C>(x[n.zp]) - xc) - L.zl * (xc - static_cast<C>(x[n.zm]));
}

// one partial sum per block and quantity, in a fixed order
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double (*sm)[BLOCK / 64],
                                               double *part, size_t pstride)
{
    const int lane = threadIdx.x + BX * threadIdx.y;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double x = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            x += __shfl_xor(x, o, 64);
        if ((lane & 63) == 0)
            sm[q][lane >> 6] = x;
    }
    __syncthreads();
    if (lane == 0) {
        const size_t blin =
            blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            // pairwise over the waves, in a fixed order
            double t[BLOCK / 64];
#pragma unroll
            for (int w = 0; w < BLOCK / 64; ++w)
                t[w] = sm[q][w];
#pragma unroll
            for (int w = BLOCK / 64; w > 1; w /= 2)
#pragma unroll
                for (int i = 0; i < w / 2; ++i)
                    t[i] = t[2 * i] + t[2 * i + 1];
            part[(size_t)q * pstride + blin] = t[0];
        }
    }
}

// Workgroups are dispatched to the 8 XCDs in turn and each XCD has its own L2.
// The stencil kernels with 2 x 2 cells per thread take their blocks in groups
// of all x-blocks of two block rows, one group per XCD in turn: the halo lines
// and rows the blocks of a group share (and the periodic wrap in x) then sit
// in one L2, while the XCDs still work through neighbouring groups, so their
// accesses stay spread over the address space.  Identity where the grid does
// not divide into such groups.
__device__ __forceinline__ void xcd_groups(unsigned &bx, unsigned &by, unsigned &bz)
{
    const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    bx = blockIdx.x;
    by = blockIdx.y;
    bz = blockIdx.z;
    if (gy % 2 != 0 || (gx * gy * gz) % 8 != 0 || ((gy / 2) * gz) % 8 != 0)
        return;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned xcd = p & 7u, slot = p >> 3;
    const unsigned member = slot % (2 * gx), group = (slot / (2 * gx)) * 8 + xcd;
    bz = group / (gy / 2);
    by = 2 * (group % (gy / 2)) + member / gx;
    bx = member % gx;
}

// The restriction takes its blocks in eighths of the whole grid instead, one
// contiguous range of block planes per XCD (where the block count divides by
// 8), so that each XCD's L2 holds a slab with halo planes at its two ends
// only; for the restriction this is the faster order, for the direction and
// residual passes the grouped one.  Identity otherwise.
__device__ __forceinline__ void xcd_slabs(unsigned &bx, unsigned &by, unsigned &bz)
{
    const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    bx = blockIdx.x;
    by = blockIdx.y;
    bz = blockIdx.z;
    const unsigned n = gx * gy * gz;
    if (n % 8 != 0)
        return;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned q = (p & 7u) * (n >> 3) + (p >> 3);
    bx = q % gx;
    by = (q / gx) % gy;
    bz = q / (gx * gy);
}

// ---------------------------------------------------------------------------
// V-cycle kernels (templated on the storage type)
// ---------------------------------------------------------------------------

// One colour of red-black Gauss-Seidel (eq. beta_pressure with relaxation 1):
// e_c <- (sum beta e_nb - h^2 r_c) / sum beta.  ZERO: e is zero on entry.
template <typename T, bool ZERO>
__global__ __launch_bounds__(BLOCK) void k_rbgs(Dims d, Bc bc, const T *__restrict__ bx,
                                                const T *__restrict__ by,
                                                const T *__restrict__ bz,
                                                const T *__restrict__ r, T *e,
                                                const T *__restrict__ sg,
                                                typename Acc<T>::type h2,
                                                typename Acc<T>::type om, int colour,
                                                int self_zero)
{
    using C = typename Acc<T>::type;
    const int t = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (j >= d.ny)
        return;
    const int i = 2 * t + ((j + k + colour) & 1);
    if (i >= d.nx)
        return;
    const Nb n = neighbours(d, bc, i, j, k);
    const Links<T> L = links(n, bx, by, bz);
    C diag = (L.xl + L.xh) + (L.yl + L.yh) + (L.zl + L.zh);
    if (sg)
        diag += ld(sg, n.c);        // h^2 sigma: the general operator's diagonal term
    C s = C(0);
    if (!ZERO) {
        s = L.xl * ld(e, n.xm) + L.xh * ld(e, n.xp) + L.yl * ld(e, n.ym) + L.yh * ld(e, n.yp) +
            L.zl * ld(e, n.zm) + L.zh * ld(e, n.zp);
    }
    // over-relaxed (eq. beta_pressure); a cell with no open face and no
    // diagonal term is excluded: it stays 0
    const C g = (s - h2 * ld(r, n.c)) / diag;
    const C v = (ZERO || self_zero) ? om * g : (C(1) - om) * ld(e, n.c) + om * g;
    e[n.c] = static_cast<T>(diag > C(0) ? v : C(0));
}

// rH = mean over the 8 children of (r - A e).  One thread per coarse column
// (I, J) walks kz coarse planes along z; the two x-children of each of its two
// child rows are handled as a pair with two-element vector loads.  The fine
// planes below and at the current one (e) and the low z-face coefficient are
// carried in registers, and the two child rows are each other's y-neighbours,
// so only the rows 2J-1 and 2J+2 and the next plane are loaded beside the
// children themselves.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_resid_restrict(Dims fd, Bc bc, const T *__restrict__ bx,
                                                          const T *__restrict__ by,
                                                          const T *__restrict__ bz,
                                                          const T *__restrict__ e,
                                                          const T *__restrict__ r,
                                                          const T *__restrict__ sg,
                                                          T *__restrict__ rH,
                                                          typename Acc<T>::type ih2, int kz)
{
    using C = typename Acc<T>::type;
    using T2 = typename Vec2<T>::type;
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    unsigned gbx, gby, gbz;
    xcd_slabs(gbx, gby, gbz);
    const int I = (int)gbx * BX + threadIdx.x;
    const int J = (int)gby * BY + threadIdx.y;
    const int K0 = (int)gbz * kz;
    const int K1 = min(K0 + kz, cd.nz);
    if (I >= cd.nx || J >= cd.ny)
        return;
    const size_t sy = (size_t)fd.nx, sz = (size_t)fd.nx * fd.ny;
    const int x = 2 * I;
    const int xm1 = (x == 0) ? fd.nx - 1 : x - 1;
    const int xp2 = (x + 2 == fd.nx) ? 0 : x + 2;
    const bool wxl = bc.x && x == 0, wxh = bc.x && x + 2 == fd.nx;
    // child rows j0 = 2J, j1 = 2J + 1 (ny is even, so j0 never touches the
    // high wall and j1 never the low one); the rows outside them
    const int j0 = 2 * J, j1 = j0 + 1;
    const int jm = (j0 == 0) ? fd.ny - 1 : j0 - 1, jp = (j1 == fd.ny - 1) ? 0 : j1 + 1;
    const bool wyl = bc.y && j0 == 0, wyh = bc.y && j1 == fd.ny - 1;
    const size_t r0 = (size_t)j0 * sy + x, r1 = (size_t)j1 * sy + x;
    auto ld2 = [](const T *p, size_t i) -> T2 { return *reinterpret_cast<const T2 *>(p + i); };
    // one fine cell pair of a child row: h^2 (A e) of both cells
    auto pair_flux = [&](T2 ec, T2 xx, C exm, C exp, C bxn, T2 ylo, T2 yhi, T2 eym, T2 eyp,
                         T2 zlo, T2 zhi, T2 ezm, T2 ezp, bool wyl_, bool wyh_, bool wzl, bool wzh,
                         C &f0, C &f1) {
        const C e0 = C(ec.x), e1 = C(ec.y);
        f0 = C(xx.y) * (e1 - e0) - (wxl ? C(0) : C(xx.x)) * (e0 - exm) +
             (wyh_ ? C(0) : C(yhi.x)) * (C(eyp.x) - e0) - (wyl_ ? C(0) : C(ylo.x)) * (e0 - C(eym.x)) +
             (wzh ? C(0) : C(zhi.x)) * (C(ezp.x) - e0) - (wzl ? C(0) : C(zlo.x)) * (e0 - C(ezm.x));
        f1 = (wxh ? C(0) : bxn) * (exp - e1) - C(xx.y) * (e1 - e0) +
             (wyh_ ? C(0) : C(yhi.y)) * (C(eyp.y) - e1) - (wyl_ ? C(0) : C(ylo.y)) * (e1 - C(eym.y)) +
             (wzh ? C(0) : C(zhi.y)) * (C(ezp.y) - e1) - (wzl ? C(0) : C(zlo.y)) * (e1 - C(ezm.y));
    };
    // the fine plane below the first one, the first one, its low z faces
    int k = 2 * K0;
    size_t pl = (size_t)k * sz;
    const size_t pm = (size_t)(k == 0 ? fd.nz - 1 : k - 1) * sz;
    T2 em0 = ld2(e, pm + r0), em1 = ld2(e, pm + r1);
    T2 ec0 = ld2(e, pl + r0), ec1 = ld2(e, pl + r1);
    T2 zl0 = ld2(bz, pl + r0), zl1 = ld2(bz, pl + r1);
    for (int K = K0; K < K1; ++K) {
        C acc = C(0);
#pragma unroll
        for (int dk = 0; dk < 2; ++dk, ++k) {
            pl = (size_t)k * sz;
            const size_t pp = (size_t)(k == fd.nz - 1 ? 0 : k + 1) * sz;
            const bool wzl = bc.z && k == 0, wzh = bc.z && k == fd.nz - 1;
            const T2 ep0 = ld2(e, pp + r0), ep1 = ld2(e, pp + r1);
            const T2 zh0 = ld2(bz, pp + r0), zh1 = ld2(bz, pp + r1);
            const T2 rr0 = ld2(r, pl + r0), rr1 = ld2(r, pl + r1);
            const T2 xx0 = ld2(bx, pl + r0), xx1 = ld2(bx, pl + r1);
            const T2 yl0 = ld2(by, pl + r0), yl1 = ld2(by, pl + r1);
            const T2 yh1 = ld2(by, pl + (size_t)jp * sy + x);
            const T2 eym = ld2(e, pl + (size_t)jm * sy + x), eyp = ld2(e, pl + (size_t)jp * sy + x);
            const size_t rw0 = pl + (size_t)j0 * sy, rw1 = pl + (size_t)j1 * sy;
            const C exm0 = ld(e, rw0 + xm1), exp0 = ld(e, rw0 + xp2);
            const C exm1 = ld(e, rw1 + xm1), exp1 = ld(e, rw1 + xp2);
            const C bxn0 = ld(bx, rw0 + xp2), bxn1 = ld(bx, rw1 + xp2);
            C f00, f01, f10, f11;
            // row j0: its high y neighbour is row j1; row j1: its low one is j0
            pair_flux(ec0, xx0, exm0, exp0, bxn0, yl0, yl1, eym, ec1, zl0, zh0, em0, ep0, wyl,
                      false, wzl, wzh, f00, f01);
            pair_flux(ec1, xx1, exm1, exp1, bxn1, yl1, yh1, ec0, eyp, zl1, zh1, em1, ep1, false,
                      wyh, wzl, wzh, f10, f11);
            // r - A e; the general operator's diagonal term sg = h^2 sigma
            // adds + sigma e = ih2 sg e
            C s00 = C(0), s01 = C(0), s10 = C(0), s11 = C(0);
            if (sg) {
                const T2 sv0 = ld2(sg, pl + r0), sv1 = ld2(sg, pl + r1);
                s00 = ih2 * (C(sv0.x) * C(ec0.x));
                s01 = ih2 * (C(sv0.y) * C(ec0.y));
                s10 = ih2 * (C(sv1.x) * C(ec1.x));
                s11 = ih2 * (C(sv1.y) * C(ec1.y));
            }
            acc += (C(rr0.x) - ih2 * f00 + s00) + (C(rr0.y) - ih2 * f01 + s01);
            acc += (C(rr1.x) - ih2 * f10 + s10) + (C(rr1.y) - ih2 * f11 + s11);
            em0 = ec0;
            em1 = ec1;
            ec0 = ep0;
            ec1 = ep1;
            zl0 = zh0;
            zl1 = zh1;
        }
        rH[((size_t)K * cd.ny + J) * cd.nx + I] = static_cast<T>(acc * C(0.125));
    }
}

__device__ __forceinline__ int other_parent(int i, int nH, int wall)
{
    const int I = i >> 1;
    int o = (i & 1) ? I + 1 : I - 1;
    if (o < 0 || o >= nH)
        o = wall ? I : (o + nH) % nH;
    return o;
}

// Weight of the far coarse cell in the prolongation of one fine cell along
// one axis.  The fine cell lies between its parent's centre (at the face
// between the two children) and the far coarse neighbour's centre (at the
// face beyond the cell's other side); along a row of links this interval is
// half a link to the parent's centre (coefficient gn: the face between the
// children), the cell's outer face (gm) and half of the link beyond it (gf).
// The weight is the near half-link's share of the series resistance,
//   w = (1/2 gn) / (1/2 gn + 1/gm + 1/2 gf) = gm gf / (gm gf + gn (2 gf + gm)),
// 1/4 for equal coefficients (trilinear interpolation), near 0 for a fine cell
// tied to its parent by a strong link and to the far cell through weak ones,
// 0 at a wall (gm = 0), and 0 for a cell closed on both sides.
__device__ __forceinline__ double far_weight(double gn, double gm, double gf)
{
    // the same bits at every call site: no contraction into fused multiply-adds
#pragma clang fp contract(off)
    const double den = gm * gf + gn * (2.0 * gf + gm);
    return den > 0.0 ? (gm * gf) / den : 0.0;
}

// The three weights of a cell are stored as 8-bit fractions of 256 in one
// 32-bit word (x in bits 0-7, y in 8-15, z in 16-23): q = round(256 w),
// at most 255, so 1/4 is exact.
__device__ __forceinline__ unsigned weight_q(double w)
{
    const int q = (int)(w * 256.0 + 0.5);
    return (unsigned)(q > 255 ? 255 : q);
}

__device__ __forceinline__ unsigned pack_weights(double wx, double wy, double wz)
{
    return weight_q(wx) | (weight_q(wy) << 8) | (weight_q(wz) << 16);
}

// The prolongation weights of the 8 fine cells of a coarse cell (x = 2I,
// y = 2J, z = 2K), stored as four x-pairs of packed words.  For each of the
// 4 rows of each axis (x: rows (dk, dj); y: columns (dk, di); z: columns
// (dj, di)) the faces x-1 .. x+3 along it: lo, mid, hi (as for
// coarse_face) and f2, f3 (the faces beyond the high child).
__device__ __forceinline__ void children_weights(const double xlo[4], const double xmid[4],
                                                 const double xhi[4], const double x2[4],
                                                 const double x3[4], const double ylo[4],
                                                 const double ymid[4], const double yhi[4],
                                                 const double y2[4], const double y3[4],
                                                 const double zlo[4], const double zmid[4],
                                                 const double zhi[4], const double z2[4],
                                                 const double z3[4], unsigned *w, size_t c00,
                                                 size_t fy, size_t fz)
{
    using U2 = unsigned __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj) {
            unsigned q[2];
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                const int rx = 2 * dk + dj, ry = 2 * dk + di, rz = 2 * dj + di;
                const double wx = di ? far_weight(xhi[rx], x2[rx], x3[rx])
                                     : far_weight(xhi[rx], xmid[rx], xlo[rx]);
                const double wy = dj ? far_weight(yhi[ry], y2[ry], y3[ry])
                                     : far_weight(yhi[ry], ymid[ry], ylo[ry]);
                const double wz = dk ? far_weight(zhi[rz], z2[rz], z3[rz])
                                     : far_weight(zhi[rz], zmid[rz], zlo[rz]);
                q[di] = pack_weights(wx, wy, wz);
            }
            *reinterpret_cast<U2 *>(w + c00 + dk * fz + dj * fy) = U2{q[0], q[1]};
        }
}

// Prolongation weights of every cell of a level, from its FP64 face
// coefficients: along each axis, an even index i (low child) has
// gn = beta[i+1], gm = beta[i], gf = beta[i-1]; an odd one gn = beta[i],
// gm = beta[i+1], gf = beta[i+2] (indices wrapped; in a wall direction the
// face of wrapped index 0, the lower wall or the implicit upper one, is 0
// whatever is stored).
__global__ __launch_bounds__(BLOCK) void k_prolong_weights(Dims d, Bc bc, const double *__restrict__ bx,
                                                           const double *__restrict__ by,
                                                           const double *__restrict__ bz,
                                                           unsigned *__restrict__ w)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny)
        return;
    const size_t sy = d.nx, sz = (size_t)d.nx * d.ny;
    const size_t c = (size_t)k * sz + (size_t)j * sy + i;
    // coefficient of face v (wrapped) along one axis
    auto face = [](const double *b, int v, int n, size_t stride, size_t base, int wall) {
        v = v < 0 ? v + n : (v >= n ? v - n : v);
        return (wall && v == 0) ? 0.0 : b[base + (size_t)v * stride];
    };
    // the weight from the faces idx-1 .. idx+2 along one axis
    auto axis = [&](const double *b, int idx, int n, size_t stride, size_t base, int wall) {
        const double f0 = face(b, idx - 1, n, stride, base, wall);
        const double f1 = face(b, idx, n, stride, base, wall);
        const double f2 = face(b, idx + 1, n, stride, base, wall);
        const double f3 = face(b, idx + 2, n, stride, base, wall);
        return (idx & 1) ? far_weight(f1, f2, f3) : far_weight(f2, f1, f0);
    };
    w[c] = pack_weights(axis(bx, i, d.nx, 1, c - i, bc.x),
                        axis(by, j, d.ny, sy, c - (size_t)j * sy, bc.y),
                        axis(bz, k, d.nz, sz, c - (size_t)k * sz, bc.z));
}

// e += P eH: cell-centred interpolation per axis between the parent and the
// next coarse cell on the fine cell's side (at a wall: the parent itself),
// the next cell weighted by the fine cell's weight w along that axis and the
// parent by 1 - w; the axes compose as a product (trilinear when every
// weight is 1/4; w null: 1/4 everywhere).  One thread per coarse cell updates
// its 2 x 2 x 2 children: it reads the 3 x 3 x 3 coarse neighbourhood once
// and adds to the children as four x-pairs (vector read-modify-write).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_prolong(Dims fd, Bc bc, const T *__restrict__ eH,
                                                   T *__restrict__ e,
                                                   const unsigned *__restrict__ w)
{
    using C = typename Acc<T>::type;
    using T2 = typename Vec2<T>::type;
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const int I = blockIdx.x * BX + threadIdx.x;
    const int J = blockIdx.y * BY + threadIdx.y;
    const int K = blockIdx.z;
    if (I >= cd.nx || J >= cd.ny)
        return;
    // the other parent of the low (0) and high (1) child along each axis
    const int In[2] = {other_parent(2 * I, cd.nx, bc.x), other_parent(2 * I + 1, cd.nx, bc.x)};
    const int Jn[2] = {other_parent(2 * J, cd.ny, bc.y), other_parent(2 * J + 1, cd.ny, bc.y)};
    const int Kn[2] = {other_parent(2 * K, cd.nz, bc.z), other_parent(2 * K + 1, cd.nz, bc.z)};
    const size_t sy = cd.nx, sz = (size_t)cd.nx * cd.ny;
    // coarse values: [z: K, Kn0, Kn1][y: J, Jn0, Jn1][x: I, In0, In1]
    C V[3][3][3];
    const int ks[3] = {K, Kn[0], Kn[1]}, js[3] = {J, Jn[0], Jn[1]}, is[3] = {I, In[0], In[1]};
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const size_t r0 = (size_t)ks[u] * sz + (size_t)js[v] * sy;
#pragma unroll
            for (int t = 0; t < 3; ++t)
                V[u][v][t] = ld(eH, r0 + is[t]);
        }
    const C q = C(0.25);
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const size_t c = ((size_t)(2 * K + cz) * fd.ny + (2 * J + cy)) * fd.nx + 2 * I;
            C ax[2] = {q, q}, ay[2] = {q, q}, az[2] = {q, q};
            if (w) {
                const U2 pw = *reinterpret_cast<const U2 *>(w + c);
                const unsigned wv[2] = {pw.x, pw.y};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    ax[h] = C(wv[h] & 255u) * C(1.0 / 256.0);
                    ay[h] = C((wv[h] >> 8) & 255u) * C(1.0 / 256.0);
                    az[h] = C((wv[h] >> 16) & 255u) * C(1.0 / 256.0);
                }
            }
            T2 *ep = reinterpret_cast<T2 *>(e + c);
            T2 ev = *ep;
            C v[2];
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                // along x in the four coarse rows (z: parent / next, y: parent / next)
                auto xl = [&](int u, int w_) {
                    return V[u][w_][0] + ax[cx] * (V[u][w_][1 + cx] - V[u][w_][0]);
                };
                const C y0 = xl(0, 0) + ay[cx] * (xl(0, 1 + cy) - xl(0, 0));
                const C y1 = xl(1 + cz, 0) + ay[cx] * (xl(1 + cz, 1 + cy) - xl(1 + cz, 0));
                v[cx] = y0 + az[cx] * (y1 - y0);
            }
            ev.x = static_cast<T>(C(ev.x) + v[0]);
            ev.y = static_cast<T>(C(ev.y) + v[1]);
            *ep = ev;
        }
    }
}

// Coarsest level: e = A^+ r with the FP64 pseudo-inverse (symmetric, n <= 1024).
template <typename T>
__global__ __launch_bounds__(1024) void k_coarsest(int n, const double *__restrict__ pinv,
                                                   const T *__restrict__ r, T *__restrict__ e)
{
    __shared__ double rs[1024];
    for (int t = threadIdx.x; t < n; t += blockDim.x)
        rs[t] = static_cast<double>(r[t]);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double s = 0.0;
        for (int jj = 0; jj < n; ++jj)
            s += pinv[(size_t)jj * n + i] * rs[jj];
        e[i] = static_cast<T>(s);
    }
}

// ---------------------------------------------------------------------------
// The bottom of the V-cycle in one workgroup.  Levels of at most a few
// thousand cells cost a kernel launch per step and little else, so all of
// them (smoothing, transfers and the coarsest solve) run in a single
// 1024-thread workgroup that walks the levels with barriers between steps.
// The arithmetic is the same as in the per-level kernels.
// ---------------------------------------------------------------------------
template <typename T>
struct TailArgs {
    int n;                     // levels in the tail (the last is the coarsest)
    Dims d[TAIL_MAX];
    double h2[TAIL_MAX];
    const T *b[TAIL_MAX][3];
    T *e[TAIL_MAX];
    T *r[TAIL_MAX];
    const T *s[TAIL_MAX];      // diagonal term of the general operator, or null
    const unsigned *w[TAIL_MAX];   // prolongation weights of each level but the last, or null
    Bc bc;
    int nu_pre, nu_post;
    double omega;              // the smoother's over-relaxation
    const double *pinv;        // pseudo-inverse of the coarsest operator
    int ncoarse;
    int warm;                  // e[0] holds a correction to start the first level from
};

// Tail levels live in LDS: corrections and right-hand sides always, face
// coefficients too when the arithmetic is FP32 (for FP64 they are read from
// global memory, where they stay in L2).  Level q occupies cells
// [off[q], off[q] + cells(d[q])) of each array.
constexpr int TAIL_LDS = 4736;            // >= 4096 * (1 + 1/8 + 1/64 + ...)
constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_PAIRS = 2;             // x-pairs per thread: 4096 cells / 2 / 1024
constexpr int TAIL_PINV = 4096;           // coarsest pseudo-inverses of up to 64 cells are staged in LDS

// One x-pair (cells i0, i0+1 of a row) of a smoothed tail level, as a thread
// holds it during a visit of that level: LDS indices of the pair and of its
// neighbours (level-relative, wraps resolved), the face coefficients with
// walls zeroed, the right-hand side and the diagonal.
template <typename C>
struct TPair {
    int c;                     // first cell
    int xm, xp;                // the cell left of the pair, the cell right of it
    int ym, yp, zm, zp;        // offsets of the y and z neighbours (the same for both cells)
    int par;                   // colour of the first cell: (j + k) & 1
    bool on;
    C fx0, fx1, fx2;           // x faces: low of cell 0, between the cells, high of cell 1
    C fyl[2], fyh[2], fzl[2], fzh[2];
    C r[2], sg[2];
    C dg[2];                   // sum of the face coefficients + h^2 sigma
};

template <typename C, typename TB, typename TS>
__device__ __forceinline__ void tp_load(TPair<C> &P, Dims d, Bc bc, int p, const TB *bx,
                                        const TB *by, const TB *bz, const C *R, const TS *sg,
                                        C h2)
{
    const int hx = d.nx / 2;
    const int npairs = hx * d.ny * d.nz;
    P.on = p < npairs;
    if (!P.on)
        p = 0;
    const int k = p / (hx * d.ny);
    const int rem = p - k * hx * d.ny;
    const int j = rem / hx;
    const int i0 = 2 * (rem - j * hx);
    const int nxy = d.nx * d.ny;
    const int c = (k * d.ny + j) * d.nx + i0;
    P.c = c;
    P.par = (j + k) & 1;
    P.xm = i0 == 0 ? c + d.nx - 1 : c - 1;
    P.xp = i0 + 2 == d.nx ? c + 2 - d.nx : c + 2;
    P.ym = j == 0 ? (d.ny - 1) * d.nx : -d.nx;
    P.yp = j == d.ny - 1 ? -(d.ny - 1) * d.nx : d.nx;
    P.zm = k == 0 ? (d.nz - 1) * nxy : -nxy;
    P.zp = k == d.nz - 1 ? -(d.nz - 1) * nxy : nxy;
    const bool wxl = bc.x && i0 == 0, wxh = bc.x && i0 + 2 == d.nx;
    const bool wyl = bc.y && j == 0, wyh = bc.y && j == d.ny - 1;
    const bool wzl = bc.z && k == 0, wzh = bc.z && k == d.nz - 1;
    P.fx0 = wxl ? C(0) : C(bx[c]);
    P.fx1 = C(bx[c + 1]);
    P.fx2 = wxh ? C(0) : C(bx[P.xp]);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        P.fyl[q] = wyl ? C(0) : C(by[c + q]);
        P.fyh[q] = wyh ? C(0) : C(by[c + q + P.yp]);
        P.fzl[q] = wzl ? C(0) : C(bz[c + q]);
        P.fzh[q] = wzh ? C(0) : C(bz[c + q + P.zp]);
        P.r[q] = R[c + q];
        P.sg[q] = sg ? C(sg[c + q]) : C(0);
    }
    P.dg[0] = (P.fx0 + P.fx1) + (P.fyl[0] + P.fyh[0]) + (P.fzl[0] + P.fzh[0]);
    P.dg[1] = (P.fx1 + P.fx2) + (P.fyl[1] + P.fyh[1]) + (P.fzl[1] + P.fzh[1]);
    if (sg) {                  // h^2 sigma, the general operator's diagonal term
        P.dg[0] += P.sg[0];
        P.dg[1] += P.sg[1];
    }
}

// Over-relaxed Gauss-Seidel update of the cell of colour `colour` in the pair
// (eq. beta_pressure, relaxation om); zero: e is zero on entry (neither the
// cell nor its neighbours are read); self_zero: the cell's own old value is
// zero (the second colour of the first sweep), its neighbours are read.
template <typename C>
__device__ __forceinline__ void tp_gs(const TPair<C> &P, C *E, C h2, C om, int colour, bool zero,
                                      bool self_zero)
{
    if (!P.on)
        return;
    const int q = colour == P.par ? 0 : 1;
    const int c = P.c + q;
    const C xl = q == 0 ? P.fx0 : P.fx1, xh = q == 0 ? P.fx1 : P.fx2;
    C s = C(0);
    if (!zero)
        s = xl * E[q == 0 ? P.xm : P.c] + xh * E[q == 0 ? P.c + 1 : P.xp] + P.fyl[q] * E[c + P.ym] +
            P.fyh[q] * E[c + P.yp] + P.fzl[q] * E[c + P.zm] + P.fzh[q] * E[c + P.zp];
    const C g = (s - h2 * P.r[q]) / P.dg[q];
    const C v = (zero || self_zero) ? om * g : (C(1) - om) * E[c] + om * g;
    // a cell with no open face and no diagonal term is excluded: it stays 0
    E[c] = P.dg[q] > C(0) ? v : C(0);
}

// r - A e at the two cells of the pair, summed (the restriction adds four pairs)
template <typename C>
__device__ __forceinline__ C tp_residual_sum(const TPair<C> &P, const C *E, C ih2)
{
    C acc = C(0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int c = P.c + q;
        const C xl = q == 0 ? P.fx0 : P.fx1, xh = q == 0 ? P.fx1 : P.fx2;
        const C ec = E[c];
        const C exm = E[q == 0 ? P.xm : P.c], exp = E[q == 0 ? P.c + 1 : P.xp];
        const C fl = xh * (exp - ec) - xl * (ec - exm) + P.fyh[q] * (E[c + P.yp] - ec) -
                     P.fyl[q] * (ec - E[c + P.ym]) + P.fzh[q] * (E[c + P.zp] - ec) -
                     P.fzl[q] * (ec - E[c + P.zm]);
        acc += P.r[q] - ih2 * fl + ih2 * (P.sg[q] * ec);
    }
    return acc;
}

// e += P eH on the pair's two cells (the interpolation of k_prolong, with the
// level's weights; w null: 1/4)
template <typename C>
__device__ __forceinline__ void tp_prolong(const TPair<C> &P, Dims fd, Bc bc, const C *EH, C *E,
                                           const unsigned *w)
{
    if (!P.on)
        return;
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const int nxy = fd.nx * fd.ny;
    const int k = P.c / nxy, rem = P.c - k * nxy;
    const int j = rem / fd.nx, i0 = rem - j * fd.nx;
    const int I = i0 >> 1;
    const int In[2] = {other_parent(i0, cd.nx, bc.x), other_parent(i0 + 1, cd.nx, bc.x)};
    const int J0 = j >> 1, J1 = other_parent(j, cd.ny, bc.y);
    const int K0 = k >> 1, K1 = other_parent(k, cd.nz, bc.z);
    const int sy = cd.nx, sz = cd.nx * cd.ny;
    const int rows[4] = {K0 * sz + J0 * sy, K0 * sz + J1 * sy, K1 * sz + J0 * sy, K1 * sz + J1 * sy};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const unsigned pw = w ? w[P.c + q] : 0x404040u;   // 64/256 = 1/4 on each axis
        const C ax = C(pw & 255u) * C(1.0 / 256.0);
        const C ay = C((pw >> 8) & 255u) * C(1.0 / 256.0);
        const C az = C((pw >> 16) & 255u) * C(1.0 / 256.0);
        C xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const C cI = EH[rows[u] + I];
            xv[u] = cI + ax * (EH[rows[u] + In[q]] - cI);
        }
        const C y0 = xv[0] + ay * (xv[1] - xv[0]);
        const C y1 = xv[2] + ay * (xv[3] - xv[2]);
        E[P.c + q] += y0 + az * (y1 - y0);
    }
}

template <typename T>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_cycle(TailArgs<T> a)
{
    using C = typename Acc<T>::type;
    constexpr bool BLDS = sizeof(C) == 4;   // FP32 arithmetic: face coefficients in LDS too
    constexpr int SPW = (TAIL_LDS / 2 * (int)sizeof(C) + 7) / 8;
    static_assert(SPW >= 1024, "the coarsest right-hand side reuses the pair sums' storage");
    static_assert(TAIL_CELLS % TAIL_THREADS == 0 && TAIL_PINV % TAIL_THREADS == 0, "staging");
    __shared__ C E[TAIL_LDS];
    __shared__ C Rr[TAIL_LDS];
    __shared__ C Bs[BLDS ? 3 : 1][BLDS ? TAIL_LDS : 1];
    __shared__ unsigned Wl[TAIL_LDS];      // prolongation weights of every level but the last
    __shared__ double Pv[TAIL_PINV];       // the coarsest pseudo-inverse, when it fits
    // per-pair residual sums during the restrictions, then the coarsest
    // right-hand side (the last restriction has finished reading the sums)
    __shared__ double SpRaw[SPW];
    C *Sp = reinterpret_cast<C *>(SpRaw);
    double *rs = SpRaw;
    const int L = a.n;
    const int tid = threadIdx.x;
    const C om = static_cast<C>(a.omega);
    int off[TAIL_MAX + 1];                  // first cell of level q in the LDS arrays
    off[0] = 0;
    for (int l = 0; l < L; ++l)
        off[l + 1] = off[l] + (int)cells(a.d[l]);
    // Stage the input right-hand side, the coefficients, the weights and a
    // small pseudo-inverse.  Every load is issued before the first LDS store,
    // so the staging costs one memory round trip.  The first level has at
    // most TAIL_CELLS cells (a fixed count per thread, indices clamped so that
    // every load is in range); the levels below it together hold fewer than
    // an eighth as many, at most one cell per thread.
    constexpr int U0 = TAIL_CELLS / TAIL_THREADS;
    constexpr int UP = TAIL_PINV / TAIL_THREADS;
    const int n0 = off[1];
    const int nrest = off[L] - n0;
    const int nwt = off[L - 1];             // weights: every level but the last
    const int nc = a.ncoarse;
    const bool pvl = nc * nc <= TAIL_PINV;
    const unsigned WDEF = 0x404040u;        // 64/256 = 1/4 on each axis: trilinear
    C r0[U0], b0[3][U0], b1[3] = {C(0), C(0), C(0)}, e0[U0];
    unsigned w0[U0], w1 = WDEF;
    double pv[UP];
    const unsigned *wf = L > 1 ? a.w[0] : nullptr;
#pragma unroll
    for (int u = 0; u < U0; ++u) {
        const int cc = min(tid + u * TAIL_THREADS, n0 - 1);
        r0[u] = ld(a.r[0], cc);
        e0[u] = a.warm ? ld(a.e[0], cc) : C(0);
#pragma unroll
        for (int m = 0; m < 3; ++m)
            b0[m][u] = BLDS ? ld(a.b[0][m], cc) : C(0);
        w0[u] = wf ? wf[cc] : WDEF;
    }
    // this thread's cell of the levels below the first: its level's arrays
    // are picked by selects over the (uniform) argument pointers, so that no
    // load waits for another
    const int g = n0 + tid;
    const T *pb[3] = {nullptr, nullptr, nullptr};
    const unsigned *pw = nullptr;
    int ob = 0;
#pragma unroll
    for (int q = 1; q < TAIL_MAX; ++q)
        if (q < L && g >= off[q]) {
#pragma unroll
            for (int m = 0; m < 3; ++m)
                pb[m] = a.b[q][m];
            pw = a.w[q];
            ob = off[q];
        }
    const bool rin = tid < nrest;
    const bool win = rin && g < nwt;
    if (rin) {
        if (BLDS)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                b1[m] = ld(pb[m], g - ob);
        if (win && pw)
            w1 = pw[g - ob];
    }
#pragma unroll
    for (int u = 0; u < UP; ++u) {
        const int i = tid + u * TAIL_THREADS;
        pv[u] = pvl ? a.pinv[min(i, nc * nc - 1)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U0; ++u) {
        const int cc = tid + u * TAIL_THREADS;
        if (cc < n0) {
            Rr[cc] = r0[u];
            if (a.warm)
                E[cc] = e0[u];
            if (BLDS)
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    Bs[BLDS ? m : 0][BLDS ? cc : 0] = b0[m][u];
            if (L > 1)
                Wl[cc] = w0[u];
        }
    }
    if (rin) {
        if (BLDS)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                Bs[BLDS ? m : 0][BLDS ? g : 0] = b1[m];
        if (win)
            Wl[g] = w1;
    }
    if (pvl)
#pragma unroll
        for (int u = 0; u < UP; ++u)
            if (tid + u * TAIL_THREADS < nc * nc)
                Pv[tid + u * TAIL_THREADS] = pv[u];
    __syncthreads();
    TPair<C> P[TAIL_PAIRS];
    auto visit = [&](int l) {
#pragma unroll
        for (int u = 0; u < TAIL_PAIRS; ++u) {
            const C h2 = (C)a.h2[l];
            if (BLDS)
                tp_load(P[u], a.d[l], a.bc, tid + u * TAIL_THREADS, &Bs[0][BLDS ? off[l] : 0],
                        &Bs[BLDS ? 1 : 0][BLDS ? off[l] : 0], &Bs[BLDS ? 2 : 0][BLDS ? off[l] : 0],
                        Rr + off[l], a.s[l], h2);
            else
                tp_load(P[u], a.d[l], a.bc, tid + u * TAIL_THREADS, a.b[l][0], a.b[l][1], a.b[l][2],
                        Rr + off[l], a.s[l], h2);
        }
    };
    for (int l = 0; l + 1 < L; ++l) {
        const C h2 = (C)a.h2[l];
        C *El = E + off[l];
        visit(l);
        for (int sw = 0; sw < a.nu_pre; ++sw)
            for (int colour = 0; colour < 2; ++colour) {
#pragma unroll
                for (int u = 0; u < TAIL_PAIRS; ++u)
                    tp_gs(P[u], El, h2, om, colour, sw == 0 && colour == 0 && !(a.warm && l == 0),
                          sw == 0 && !(a.warm && l == 0));
                __syncthreads();
            }
        // restriction: residual sums per pair, then four pairs per coarse cell
        const int np = (int)cells(a.d[l]) / 2;
#pragma unroll
        for (int u = 0; u < TAIL_PAIRS; ++u)
            if (P[u].on)
                Sp[tid + u * TAIL_THREADS] = tp_residual_sum(P[u], El, C(1) / h2);
        __syncthreads();
        const Dims fd = a.d[l];
        const int hx = fd.nx / 2;
        const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
        for (int cc = tid; cc < (int)cells(cd); cc += TAIL_THREADS) {
            const int K = cc / (cd.nx * cd.ny), rem = cc - K * cd.nx * cd.ny;
            const int J = rem / cd.nx, I = rem - J * cd.nx;
            const int p00 = ((2 * K) * fd.ny + 2 * J) * hx + I;
            const int sy = hx, sz = hx * fd.ny;
            Rr[off[l + 1] + cc] = C(0.125) * ((Sp[p00] + Sp[p00 + sy]) + (Sp[p00 + sz] + Sp[p00 + sz + sy]));
        }
        (void)np;
        __syncthreads();
    }
    // coarsest level: e = A^+ r in FP64, g threads per output reduced by shuffles
    {
        const int n = a.ncoarse;
        for (int t = tid; t < n; t += TAIL_THREADS)
            rs[t] = static_cast<double>(Rr[off[L - 1] + t]);
        __syncthreads();
        int gs = 1;
        while (gs < 64 && 2 * gs * n <= TAIL_THREADS)
            gs *= 2;
        const int outp = tid / gs, lane = tid % gs;
        double s = 0.0;
        if (outp < n) {
            if (pvl)
                for (int jj = lane; jj < n; jj += gs)
                    s += Pv[jj * n + outp] * rs[jj];
            else
                for (int jj = lane; jj < n; jj += gs)
                    s += a.pinv[(size_t)jj * n + outp] * rs[jj];
        }
        for (int o = gs >> 1; o > 0; o >>= 1)
            s += __shfl_xor(s, o, 64);
        if (lane == 0 && outp < n)
            E[off[L - 1] + outp] = static_cast<C>(s);
        __syncthreads();
    }
    for (int l = L - 2; l >= 0; --l) {
        const C h2 = (C)a.h2[l];
        C *El = E + off[l];
        visit(l);
#pragma unroll
        for (int u = 0; u < TAIL_PAIRS; ++u)
            tp_prolong(P[u], a.d[l], a.bc, E + off[l + 1], El, Wl + off[l]);
        __syncthreads();
        for (int sw = 0; sw < a.nu_post; ++sw)
            for (int colour = 1; colour >= 0; --colour) {
#pragma unroll
                for (int u = 0; u < TAIL_PAIRS; ++u)
                    tp_gs(P[u], El, h2, om, colour, false, false);
                __syncthreads();
            }
    }
    // the correction of the tail's first level goes back to global memory
    for (int c = tid; c < off[1]; c += TAIL_THREADS)
        a.e[0][c] = static_cast<T>(E[c]);
}

template <typename T>
__global__ void k_convert(size_t n, const double *__restrict__ src, T *__restrict__ dst)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = static_cast<T>(src[i]);
}

// dst = scale * src, counting (partials) the entries whose magnitude reaches
// `limit` in the storage type (FP16 range checks)
template <typename T>
__global__ __launch_bounds__(256) void k_convert_scaled(size_t n, const double *__restrict__ src,
                                                         double scale, double limit,
                                                         T *__restrict__ dst, double *part)
{
    __shared__ double sm[4];
    double over = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double v = scale * src[i];
        if (!(fabs(v) < limit))
            over += 1.0;
        dst[i] = static_cast<T>(v);
    }
    for (int o = 32; o > 0; o >>= 1)
        over += __shfl_xor(over, o, 64);
    if ((threadIdx.x & 63) == 0)
        sm[threadIdx.x >> 6] = over;
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = (sm[0] + sm[1]) + (sm[2] + sm[3]);
}

template <typename T>
__global__ void k_to_double(size_t n, const T *__restrict__ src, double *__restrict__ dst)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = static_cast<double>(src[i]);
}

// ---------------------------------------------------------------------------
// setup kernels (FP64)
// ---------------------------------------------------------------------------

// Coarse face coefficient from the 4 fine rows that cross a coarse face, each
// row given by its faces lo = 2I-1, mid = 2I and hi = 2I+1 along the normal
// (mid lies on the coarse face, lo and hi at the centres of the two coarse
// cells).  It weighs two estimates of the conductance between the two
// coarse centres, 1/4 and 3/4, with the rows in parallel: each row's conductance taken
// at the coarse face alone (exact when the coefficients vary only across the
// face; the mean of the 4 faces), and each row's links in series over the
// distance 2h (half a link, a link, half a link: exact when they vary only
// along the normal).  The first estimate overrates a face that cuts through
// a small inclusion of large coefficient, the second ignores flow between
// the rows; a closed link (0) gives a series term of 0.  The weights were
// measured: from equal weights to 1/4 and 3/4 the bubble case (20 gas bubbles,
// density ratio 1000) goes from 26 to 23 outer iterations and the layer case
// stays at 7.  Rows are summed in the order 0 + 1, 2 + 3 of the callers'
// (outer, inner) row indices.
__device__ __forceinline__ double coarse_face(const double lo[4], const double mid[4],
                                              const double hi[4])
{
    // the same bits at every call site: no contraction into fused multiply-adds
#pragma clang fp contract(off)
    double ser[4];
    // 2 / (1/(2 lo) + 1/mid + 1/(2 hi)) with one division
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double den = (mid[q] * hi[q] + 2.0 * (lo[q] * hi[q])) + lo[q] * mid[q];
        ser[q] = den > 0.0 ? (4.0 * lo[q]) * (mid[q] * hi[q]) / den : 0.0;
    }
    const double par = 0.25 * ((mid[0] + mid[1]) + (mid[2] + mid[3]));
    const double srs = 0.25 * ((ser[0] + ser[1]) + (ser[2] + ser[3]));
    return 0.25 * par + 0.75 * srs;
}

// coarse face coefficients (coarse_face) of every coarse face; wall faces stay 0
__global__ __launch_bounds__(BLOCK) void k_coarsen_beta(Dims fd, Bc bc, const double *__restrict__ bx,
                                                        const double *__restrict__ by,
                                                        const double *__restrict__ bz,
                                                        double *__restrict__ hx,
                                                        double *__restrict__ hy,
                                                        double *__restrict__ hz)
{
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const int I = blockIdx.x * BX + threadIdx.x;
    const int J = blockIdx.y * BY + threadIdx.y;
    const int K = blockIdx.z;
    if (I >= cd.nx || J >= cd.ny)
        return;
    const size_t sy = fd.nx, sz = (size_t)fd.nx * fd.ny;
    const int x = 2 * I, y = 2 * J, z = 2 * K;
    // the face below each coarse cell's low face, wrapped (only used where
    // the coarse face is not a wall)
    const int xl = (x == 0) ? fd.nx - 1 : x - 1;
    const int yl = (y == 0) ? fd.ny - 1 : y - 1;
    const int zl = (z == 0) ? fd.nz - 1 : z - 1;
    const size_t C = ((size_t)K * cd.ny + J) * cd.nx + I;
    double lo[4], mid[4], hi[4];
    // x faces: rows (k, j) in {2K, 2K+1} x {2J, 2J+1}
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj) {
            const size_t row = (size_t)(z + dk) * sz + (size_t)(y + dj) * sy;
            lo[2 * dk + dj] = bx[row + xl];
            mid[2 * dk + dj] = bx[row + x];
            hi[2 * dk + dj] = bx[row + x + 1];
        }
    hx[C] = (bc.x && I == 0) ? 0.0 : coarse_face(lo, mid, hi);
    // y faces: columns (k, i) in {2K, 2K+1} x {2I, 2I+1}
    for (int dk = 0; dk < 2; ++dk)
        for (int di = 0; di < 2; ++di) {
            const size_t col = (size_t)(z + dk) * sz + (size_t)(x + di);
            lo[2 * dk + di] = by[col + (size_t)yl * sy];
            mid[2 * dk + di] = by[col + (size_t)y * sy];
            hi[2 * dk + di] = by[col + (size_t)(y + 1) * sy];
        }
    hy[C] = (bc.y && J == 0) ? 0.0 : coarse_face(lo, mid, hi);
    // z faces: columns (j, i) in {2J, 2J+1} x {2I, 2I+1}
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            const size_t col = (size_t)(y + dj) * sy + (size_t)(x + di);
            lo[2 * dj + di] = bz[col + (size_t)zl * sz];
            mid[2 * dj + di] = bz[col + (size_t)z * sz];
            hi[2 * dj + di] = bz[col + (size_t)(z + 1) * sz];
        }
    hz[C] = (bc.z && K == 0) ? 0.0 : coarse_face(lo, mid, hi);
}

__global__ __launch_bounds__(BLOCK) void k_zero_walls(Dims d, Bc bc, double *bx, double *by, double *bz)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny)
        return;
    const size_t c = ((size_t)k * d.ny + j) * d.nx + i;
    if (bc.x && i == 0)
        bx[c] = 0.0;
    if (bc.y && j == 0)
        by[c] = 0.0;
    if (bc.z && k == 0)
        bz[c] = 0.0;
}

// Coefficient load in one pass over the fine level (all n even): copies the
// caller's beta (FP64) with wall faces set to 0, counts non-wall faces that
// are not finite positive numbers, writes the storage-precision copy used by
// the V-cycle (WT), and the first coarse level (mean of the 4 fine faces of
// each coarse face).  One thread per coarse cell, i.e. per 2x2x2 fine block;
// each block of threads covers kz coarse planes.  part null: no count (the
// coarse levels, formed from valid coefficients, load one plane per block so
// that their short grids do not walk planes in series).  htx (may be null):
// the coarse level's storage copy too.
template <typename T, bool WT>
__global__ __launch_bounds__(BLOCK) void k_load_coeffs(Dims fd, Bc bc, const double *__restrict__ sx,
                                                       const double *__restrict__ sy_,
                                                       const double *__restrict__ sz_,
                                                       double *__restrict__ dx, double *__restrict__ dy,
                                                       double *__restrict__ dz, T *__restrict__ tx,
                                                       T *__restrict__ ty, T *__restrict__ tz,
                                                       double *__restrict__ hx, double *__restrict__ hy,
                                                       double *__restrict__ hz, T *__restrict__ htx,
                                                       T *__restrict__ hty, T *__restrict__ htz,
                                                       unsigned *__restrict__ w0, double *part, int kz)
{
    using D2 = double __attribute__((ext_vector_type(2)));
    using T2 = typename Vec2<T>::type;
    __shared__ double sm[1][BLOCK / 64];
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const int I = blockIdx.x * BX + threadIdx.x;
    const int J = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (I < cd.nx && J < cd.ny) {
        const size_t fy = (size_t)fd.nx, fz = (size_t)fd.nx * fd.ny;
        const int x = 2 * I, y = 2 * J;
        // the faces 2I-1, 2J-1, 2K-1 below the coarse cell and the pairs of
        // faces from 2I+2, 2J+2, 2K+2 above it (wrapped)
        const int xl = (x == 0) ? fd.nx - 1 : x - 1;
        const int yl = (y == 0) ? fd.ny - 1 : y - 1;
        const int xu = (x + 2 == fd.nx) ? 0 : x + 2;
        const int yu = (y + 2 == fd.ny) ? 0 : y + 2, yu3 = (yu + 1 == fd.ny) ? 0 : yu + 1;
        // a face of wrapped index 0 in a wall direction is the wall (the
        // implicit upper one when reached from above): 0 whatever is stored
        const bool wxu = bc.x && xu == 0, wyu = bc.y && yu == 0;
        const int Ke = min(cd.nz, ((int)blockIdx.z + 1) * kz);
        for (int K = blockIdx.z * kz; K < Ke; ++K) {
            const int zl = (K == 0) ? fd.nz - 1 : 2 * K - 1;
            const int zu = (2 * K + 2 == fd.nz) ? 0 : 2 * K + 2, zu3 = (zu + 1 == fd.nz) ? 0 : zu + 1;
            const bool wzu = bc.z && zu == 0;
            // rows of the coarse faces, in coarse_face's order: lo, mid, hi;
            // and the two faces beyond each row's high child (weights)
            double xlo[4], xmid[4], xhi[4], ylo[4], ymid[4], yhi[4], zlo[4], zmid[4], zhi[4];
            double x2[4], x3[4], y2[4], y3[4], z2[4], z3[4];
            for (int dk = 0; dk < 2; ++dk)
                for (int dj = 0; dj < 2; ++dj) {
                    const int j = 2 * J + dj, k = 2 * K + dk;
                    const size_t c = (size_t)k * fz + (size_t)j * fy + 2 * I;
                    D2 bxv = *reinterpret_cast<const D2 *>(sx + c);
                    D2 byv = *reinterpret_cast<const D2 *>(sy_ + c);
                    D2 bzv = *reinterpret_cast<const D2 *>(sz_ + c);
                    const bool wx = bc.x && I == 0, wy = bc.y && j == 0, wz = bc.z && k == 0;
                    if (wx) bxv.x = 0.0;
                    if (wy) byv = D2{0.0, 0.0};
                    if (wz) bzv = D2{0.0, 0.0};
                    const double f[6] = {bxv.x, bxv.y, byv.x, byv.y, bzv.x, bzv.y};
                    const bool w[6] = {wx, false, wy, wy, wz, wz};
                    for (int q = 0; q < 6; ++q)
                        if (!w[q] && !(f[q] > 0.0 && f[q] < INFINITY))
                            v[0] += 1.0;
                    *reinterpret_cast<D2 *>(dx + c) = bxv;
                    *reinterpret_cast<D2 *>(dy + c) = byv;
                    *reinterpret_cast<D2 *>(dz + c) = bzv;
                    if (WT) {
                        *reinterpret_cast<T2 *>(tx + c) = T2{static_cast<T>(bxv.x), static_cast<T>(bxv.y)};
                        *reinterpret_cast<T2 *>(ty + c) = T2{static_cast<T>(byv.x), static_cast<T>(byv.y)};
                        *reinterpret_cast<T2 *>(tz + c) = T2{static_cast<T>(bzv.x), static_cast<T>(bzv.y)};
                    }
                    const size_t row = (size_t)k * fz + (size_t)j * fy;
                    xlo[2 * dk + dj] = sx[row + xl];
                    xmid[2 * dk + dj] = bxv.x;
                    xhi[2 * dk + dj] = bxv.y;
                    const D2 xb = *reinterpret_cast<const D2 *>(sx + row + xu);
                    x2[2 * dk + dj] = wxu ? 0.0 : xb.x;
                    x3[2 * dk + dj] = xb.y;
                    if (dj == 0) {
                        const D2 l = *reinterpret_cast<const D2 *>(sy_ + (size_t)k * fz +
                                                                   (size_t)yl * fy + x);
                        ylo[2 * dk] = l.x;
                        ylo[2 * dk + 1] = l.y;
                        ymid[2 * dk] = byv.x;
                        ymid[2 * dk + 1] = byv.y;
                    } else {
                        yhi[2 * dk] = byv.x;
                        yhi[2 * dk + 1] = byv.y;
                        const D2 a = *reinterpret_cast<const D2 *>(sy_ + (size_t)k * fz +
                                                                   (size_t)yu * fy + x);
                        const D2 b = *reinterpret_cast<const D2 *>(sy_ + (size_t)k * fz +
                                                                   (size_t)yu3 * fy + x);
                        y2[2 * dk] = wyu ? 0.0 : a.x;
                        y2[2 * dk + 1] = wyu ? 0.0 : a.y;
                        y3[2 * dk] = b.x;
                        y3[2 * dk + 1] = b.y;
                    }
                    if (dk == 0) {
                        const D2 l = *reinterpret_cast<const D2 *>(sz_ + (size_t)zl * fz +
                                                                   (size_t)j * fy + x);
                        zlo[2 * dj] = l.x;
                        zlo[2 * dj + 1] = l.y;
                        zmid[2 * dj] = bzv.x;
                        zmid[2 * dj + 1] = bzv.y;
                    } else {
                        zhi[2 * dj] = bzv.x;
                        zhi[2 * dj + 1] = bzv.y;
                        const D2 a = *reinterpret_cast<const D2 *>(sz_ + (size_t)zu * fz +
                                                                   (size_t)j * fy + x);
                        const D2 b = *reinterpret_cast<const D2 *>(sz_ + (size_t)zu3 * fz +
                                                                   (size_t)j * fy + x);
                        z2[2 * dj] = wzu ? 0.0 : a.x;
                        z2[2 * dj + 1] = wzu ? 0.0 : a.y;
                        z3[2 * dj] = b.x;
                        z3[2 * dj + 1] = b.y;
                    }
                }
            const size_t C = ((size_t)K * cd.ny + J) * cd.nx + I;
            // the same values in the same order as k_coarsen_beta
            const double cx = (bc.x && I == 0) ? 0.0 : coarse_face(xlo, xmid, xhi);
            const double cy = (bc.y && J == 0) ? 0.0 : coarse_face(ylo, ymid, yhi);
            const double cz = (bc.z && K == 0) ? 0.0 : coarse_face(zlo, zmid, zhi);
            hx[C] = cx;
            hy[C] = cy;
            hz[C] = cz;
            if (htx) {
                htx[C] = static_cast<T>(cx);
                hty[C] = static_cast<T>(cy);
                htz[C] = static_cast<T>(cz);
            }
            // the level's prolongation weights, as k_prolong_weights forms them
            children_weights(xlo, xmid, xhi, x2, x3, ylo, ymid, yhi, y2, y3, zlo, zmid, zhi, z2, z3,
                             w0, (size_t)(2 * K) * fz + (size_t)y * fy + x, fy, fz);
        }
    }
    if (part)
        block_partials<1>(v, sm, part, 0);
}

// k_load_coeffs with the face coefficients computed from the cell densities
// on the way (beta = 2 / (rho_L + rho_R), the expression of k_face_coeffs, so
// the bits are the same): each coarse cell's 8 children read rho at the
// children and at their low x, y, z neighbours, and copy it to rcopy, which
// the outer operator kernels read in place of the three coefficient arrays.
// dx == nullptr: the FP64 fine-level coefficients are not written (the
// caller forms them from rcopy when something needs them).
// Partial: non-wall faces whose beta is not a finite positive number plus
// cells whose rho is not.
template <typename T, bool WT>
__global__ __launch_bounds__(BLOCK) void k_load_density(Dims fd, Bc bc, const double *__restrict__ rho,
                                                        double *__restrict__ dx,
                                                        double *__restrict__ dy,
                                                        double *__restrict__ dz, T *__restrict__ tx,
                                                        T *__restrict__ ty, T *__restrict__ tz,
                                                        double *__restrict__ hx,
                                                        double *__restrict__ hy,
                                                        double *__restrict__ hz,
                                                        double *__restrict__ rcopy,
                                                        unsigned *__restrict__ w0, double *part)
{
    using D2 = double __attribute__((ext_vector_type(2)));
    using T2 = typename Vec2<T>::type;
    __shared__ double sm[1][BLOCK / 64];
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const int I = blockIdx.x * BX + threadIdx.x;
    const int J = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (I < cd.nx && J < cd.ny) {
        const size_t fy = (size_t)fd.nx, fz = (size_t)fd.nx * fd.ny;
        const int x = 2 * I, y = 2 * J;
        const int xm = (x == 0) ? fd.nx - 1 : x - 1;
        // the cells below the faces 2I-1, 2J-1 (wrapped): those faces are
        // 2 / (rho[2I-2] + rho[2I-1]) and 2 / (rho[2J-2] + rho[2J-1])
        const int xm2 = (x < 2) ? x - 2 + fd.nx : x - 2;
        const int ym2 = (y < 2) ? y - 2 + fd.ny : y - 2;
        // the cells x+2, x+3 (and rows, planes) above the coarse cell
        // (wrapped): the faces x+2 and x+3 are 2 / (rho[x+1] + rho[x+2]) and
        // 2 / (rho[x+2] + rho[x+3]); in a wall direction the face x+2 of
        // wrapped index 0 is the implicit upper wall
        const int xu = (x + 2 == fd.nx) ? 0 : x + 2;
        const int yu = (y + 2 == fd.ny) ? 0 : y + 2, yu3 = (yu + 1 == fd.ny) ? 0 : yu + 1;
        const bool wxu = bc.x && xu == 0, wyu = bc.y && yu == 0;
        const int Ke = min(cd.nz, ((int)blockIdx.z + 1) * (RZ / 2));
        for (int K = blockIdx.z * (RZ / 2); K < Ke; ++K) {
            const int z = 2 * K;
            const int zm2 = (z < 2) ? z - 2 + fd.nz : z - 2;
            const int zu = (z + 2 == fd.nz) ? 0 : z + 2, zu3 = (zu + 1 == fd.nz) ? 0 : zu + 1;
            const bool wzu = bc.z && zu == 0;
            // rows of the coarse faces, in coarse_face's order: lo, mid, hi;
            // and the two faces beyond each row's high child (weights)
            double xlo[4], xmid[4], xhi[4], ylo[4], ymid[4], yhi[4], zlo[4], zmid[4], zhi[4];
            double x2[4], x3[4], y2[4], y3[4], z2[4], z3[4];
            for (int dk = 0; dk < 2; ++dk)
                for (int dj = 0; dj < 2; ++dj) {
                    const int j = 2 * J + dj, k = 2 * K + dk;
                    const int jm = (j == 0) ? fd.ny - 1 : j - 1;
                    const int km = (k == 0) ? fd.nz - 1 : k - 1;
                    const size_t row = (size_t)k * fz + (size_t)j * fy;
                    const size_t c = row + x;
                    const D2 rc = *reinterpret_cast<const D2 *>(rho + c);
                    const double rxm = rho[row + xm];
                    const D2 rym = *reinterpret_cast<const D2 *>(rho + (size_t)k * fz + (size_t)jm * fy + x);
                    const D2 rzm = *reinterpret_cast<const D2 *>(rho + (size_t)km * fz + (size_t)j * fy + x);
                    const bool wx = bc.x && I == 0, wy = bc.y && j == 0, wz = bc.z && k == 0;
                    D2 bxv, byv, bzv;
                    bxv.x = wx ? 0.0 : 2.0 / (rxm + rc.x);
                    bxv.y = 2.0 / (rc.x + rc.y);
                    byv = wy ? D2{0.0, 0.0} : D2{2.0 / (rym.x + rc.x), 2.0 / (rym.y + rc.y)};
                    bzv = wz ? D2{0.0, 0.0} : D2{2.0 / (rzm.x + rc.x), 2.0 / (rzm.y + rc.y)};
                    const double f[6] = {bxv.x, bxv.y, byv.x, byv.y, bzv.x, bzv.y};
                    const bool w[6] = {wx, false, wy, wy, wz, wz};
                    for (int q = 0; q < 6; ++q)
                        if (!w[q] && !(f[q] > 0.0 && f[q] < INFINITY))
                            v[0] += 1.0;
                    if (!(rc.x > 0.0 && rc.x < INFINITY))
                        v[0] += 1.0;
                    if (!(rc.y > 0.0 && rc.y < INFINITY))
                        v[0] += 1.0;
                    if (dx) {
                        *reinterpret_cast<D2 *>(dx + c) = bxv;
                        *reinterpret_cast<D2 *>(dy + c) = byv;
                        *reinterpret_cast<D2 *>(dz + c) = bzv;
                    }
                    *reinterpret_cast<D2 *>(rcopy + c) = rc;
                    if (WT) {
                        *reinterpret_cast<T2 *>(tx + c) = T2{static_cast<T>(bxv.x), static_cast<T>(bxv.y)};
                        *reinterpret_cast<T2 *>(ty + c) = T2{static_cast<T>(byv.x), static_cast<T>(byv.y)};
                        *reinterpret_cast<T2 *>(tz + c) = T2{static_cast<T>(bzv.x), static_cast<T>(bzv.y)};
                    }
                    // the faces 2I-1, 2I+2 and 2I+3 of the row, as k_face_coeffs forms them
                    xlo[2 * dk + dj] = 2.0 / (rho[row + xm2] + rxm);
                    xmid[2 * dk + dj] = bxv.x;
                    xhi[2 * dk + dj] = bxv.y;
                    const D2 ru = *reinterpret_cast<const D2 *>(rho + row + xu);
                    x2[2 * dk + dj] = wxu ? 0.0 : 2.0 / (rc.y + ru.x);
                    x3[2 * dk + dj] = 2.0 / (ru.x + ru.y);
                    if (dj == 0) {
                        const D2 r2 = *reinterpret_cast<const D2 *>(rho + (size_t)k * fz +
                                                                    (size_t)ym2 * fy + x);
                        ylo[2 * dk] = 2.0 / (r2.x + rym.x);
                        ylo[2 * dk + 1] = 2.0 / (r2.y + rym.y);
                        ymid[2 * dk] = byv.x;
                        ymid[2 * dk + 1] = byv.y;
                    } else {
                        yhi[2 * dk] = byv.x;
                        yhi[2 * dk + 1] = byv.y;
                        // rc is the row y+1 here
                        const D2 a = *reinterpret_cast<const D2 *>(rho + (size_t)k * fz +
                                                                   (size_t)yu * fy + x);
                        const D2 b = *reinterpret_cast<const D2 *>(rho + (size_t)k * fz +
                                                                   (size_t)yu3 * fy + x);
                        y2[2 * dk] = wyu ? 0.0 : 2.0 / (rc.x + a.x);
                        y2[2 * dk + 1] = wyu ? 0.0 : 2.0 / (rc.y + a.y);
                        y3[2 * dk] = 2.0 / (a.x + b.x);
                        y3[2 * dk + 1] = 2.0 / (a.y + b.y);
                    }
                    if (dk == 0) {
                        const D2 r2 = *reinterpret_cast<const D2 *>(rho + (size_t)zm2 * fz +
                                                                    (size_t)j * fy + x);
                        zlo[2 * dj] = 2.0 / (r2.x + rzm.x);
                        zlo[2 * dj + 1] = 2.0 / (r2.y + rzm.y);
                        zmid[2 * dj] = bzv.x;
                        zmid[2 * dj + 1] = bzv.y;
                    } else {
                        zhi[2 * dj] = bzv.x;
                        zhi[2 * dj + 1] = bzv.y;
                        // rc is the plane z+1 here
                        const D2 a = *reinterpret_cast<const D2 *>(rho + (size_t)zu * fz +
                                                                   (size_t)j * fy + x);
                        const D2 b = *reinterpret_cast<const D2 *>(rho + (size_t)zu3 * fz +
                                                                   (size_t)j * fy + x);
                        z2[2 * dj] = wzu ? 0.0 : 2.0 / (rc.x + a.x);
                        z2[2 * dj + 1] = wzu ? 0.0 : 2.0 / (rc.y + a.y);
                        z3[2 * dj] = 2.0 / (a.x + b.x);
                        z3[2 * dj + 1] = 2.0 / (a.y + b.y);
                    }
                }
            const size_t C = ((size_t)K * cd.ny + J) * cd.nx + I;
            // the same values in the same order as k_coarsen_beta
            hx[C] = (bc.x && I == 0) ? 0.0 : coarse_face(xlo, xmid, xhi);
            hy[C] = (bc.y && J == 0) ? 0.0 : coarse_face(ylo, ymid, yhi);
            hz[C] = (bc.z && K == 0) ? 0.0 : coarse_face(zlo, zmid, zhi);
            // the level's prolongation weights, as k_prolong_weights forms them
            children_weights(xlo, xmid, xhi, x2, x3, ylo, ymid, yhi, y2, y3, zlo, zmid, zhi, z2, z3,
                             w0, (size_t)z * fz + (size_t)y * fy + x, fy, fz);
        }
    }
    block_partials<1>(v, sm, part, 0);
}

// counts cells whose density is not a finite positive number
__global__ __launch_bounds__(BLOCK) void k_check_rho(Dims d, const double *__restrict__ rho,
                                                     double *part)
{
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const double r = rho[((size_t)k * d.ny + j) * d.nx + i];
            if (!(r > 0.0 && r < INFINITY))
                v[0] += 1.0;
        }
    }
    block_partials<1>(v, sm, part, 0);
}

// counts non-wall faces whose beta is not a finite positive number
__global__ __launch_bounds__(BLOCK) void k_check_beta(Dims d, Bc bc, const double *__restrict__ bx,
                                                      const double *__restrict__ by,
                                                      const double *__restrict__ bz, int allow_zero,
                                                      double *part)
{
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const size_t c = ((size_t)k * d.ny + j) * d.nx + i;
            const double b[3] = {bx[c], by[c], bz[c]};
            const bool wall[3] = {bc.x && i == 0, bc.y && j == 0, bc.z && k == 0};
            for (int m = 0; m < 3; ++m)
                if (!wall[m] && !((allow_zero ? b[m] >= 0.0 : b[m] > 0.0) && b[m] < INFINITY))
                    v[0] += 1.0;
        }
    }
    block_partials<1>(v, sm, part, 0);
}

// General operator: partials of the count of sigma entries that are not
// finite non-negative numbers, and of the count of positive ones.
__global__ __launch_bounds__(BLOCK) void k_check_sigma(Dims d, const double *__restrict__ sg,
                                                       double *part, size_t pstride)
{
    __shared__ double sm[2][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[2] = {0.0, 0.0};
    if (i < d.nx && j < d.ny) {
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const double x = sg[((size_t)k * d.ny + j) * d.nx + i];
            if (!(x >= 0.0 && x < INFINITY))
                v[0] += 1.0;
            if (x > 0.0)
                v[1] += 1.0;
        }
    }
    block_partials<2>(v, sm, part, pstride);
}

// act[c] = 1 for a cell of the system (an open face or sigma > 0), else 0;
// partials of the count of active cells
__global__ __launch_bounds__(BLOCK) void k_active(Dims d, Bc bc, const double *__restrict__ bx,
                                                  const double *__restrict__ by,
                                                  const double *__restrict__ bz,
                                                  const double *__restrict__ sg,
                                                  unsigned char *__restrict__ act, double *part)
{
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const Nb n = neighbours(d, bc, i, j, k);
            const Links<double> L = links(n, bx, by, bz);
            const double dg = (L.xl + L.xh) + (L.yl + L.yh) + (L.zl + L.zh) + (sg ? sg[n.c] : 0.0);
            const bool a = dg > 0.0;
            act[n.c] = a ? 1 : 0;
            v[0] += a ? 1.0 : 0.0;
        }
    }
    block_partials<1>(v, sm, part, 0);
}

// coarse diagonal term = mean of the 8 children (the restriction is the mean)
__global__ __launch_bounds__(BLOCK) void k_coarsen_sigma(Dims fd, const double *__restrict__ sg,
                                                         double *__restrict__ sH)
{
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const int I = blockIdx.x * BX + threadIdx.x;
    const int J = blockIdx.y * BY + threadIdx.y;
    const int K = blockIdx.z;
    if (I >= cd.nx || J >= cd.ny)
        return;
    double acc = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj) {
            const size_t c = ((size_t)(2 * K + dk) * fd.ny + (2 * J + dj)) * fd.nx + 2 * I;
            acc += sg[c] + sg[c + 1];
        }
    sH[((size_t)K * cd.ny + J) * cd.nx + I] = 0.125 * acc;
}

// x = 0 on the excluded cells of the general operator
__global__ void k_mask(size_t n, double *__restrict__ x, const unsigned char *__restrict__ act)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        if (!act[i])
            x[i] = 0.0;
}

// beta_m[c] = 2 / (rho[c - e_m] + rho[c]); 0 on wall faces
__global__ __launch_bounds__(BLOCK) void k_face_coeffs(Dims d, Bc bc, const double *__restrict__ rho,
                                                       double *__restrict__ bx,
                                                       double *__restrict__ by,
                                                       double *__restrict__ bz)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny)
        return;
    const Nb n = neighbours(d, bc, i, j, k);
    const double rc = rho[n.c];
    bx[n.c] = (bc.x && i == 0) ? 0.0 : 2.0 / (rho[n.xm] + rc);
    by[n.c] = (bc.y && j == 0) ? 0.0 : 2.0 / (rho[n.ym] + rc);
    bz[n.c] = (bc.z && k == 0) ? 0.0 : 2.0 / (rho[n.zm] + rc);
}

// out = scale/h * sum_m (u_m(high face) - u_m(low face)), wall faces 0; with
// face coefficients given (the general operator), closed links (beta = 0)
// carry no flux either
__global__ __launch_bounds__(BLOCK) void k_divergence(Dims d, Bc bc, const double *__restrict__ ux,
                                                      const double *__restrict__ uy,
                                                      const double *__restrict__ uz, double s_h,
                                                      const double *__restrict__ bx,
                                                      const double *__restrict__ by,
                                                      const double *__restrict__ bz,
                                                      double *__restrict__ out)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny)
        return;
    const Nb n = neighbours(d, bc, i, j, k);
    double xl = n.wxl ? 0.0 : ux[n.c], xh = n.wxh ? 0.0 : ux[n.xp];
    double yl = n.wyl ? 0.0 : uy[n.c], yh = n.wyh ? 0.0 : uy[n.yp];
    double zl = n.wzl ? 0.0 : uz[n.c], zh = n.wzh ? 0.0 : uz[n.zp];
    if (bx) {
        xl = bx[n.c] == 0.0 ? 0.0 : xl;
        xh = bx[n.xp] == 0.0 ? 0.0 : xh;
        yl = by[n.c] == 0.0 ? 0.0 : yl;
        yh = by[n.yp] == 0.0 ? 0.0 : yh;
        zl = bz[n.c] == 0.0 ? 0.0 : zl;
        zh = bz[n.zp] == 0.0 ? 0.0 : zh;
    }
    out[n.c] = s_h * ((xh - xl) + (yh - yl) + (zh - zl));
}

// k_divergence for the pressure operator (no face coefficients) walking RZ
// planes per thread, which also sums the values it writes, in the blocks and
// the order of k_sum: the partials are those k_sum would form from `out`,
// bit for bit, so the right-hand side's mean needs no pass of its own
__global__ __launch_bounds__(BLOCK) void k_divergence_sum(Dims d, Bc bc,
                                                          const double *__restrict__ ux,
                                                          const double *__restrict__ uy,
                                                          const double *__restrict__ uz,
                                                          double s_h, double *__restrict__ out,
                                                          double *part)
{
    // the sum takes the rounded values, as k_sum reads them (no fused
    // multiply-add of the product into the sum)
#pragma clang fp contract(off)
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const Nb n = neighbours(d, bc, i, j, k);
            const double xl = n.wxl ? 0.0 : ux[n.c], xh = n.wxh ? 0.0 : ux[n.xp];
            const double yl = n.wyl ? 0.0 : uy[n.c], yh = n.wyh ? 0.0 : uy[n.yp];
            const double zl = n.wzl ? 0.0 : uz[n.c], zh = n.wzh ? 0.0 : uz[n.zp];
            const double val = s_h * ((xh - xl) + (yh - yl) + (zh - zl));
            out[n.c] = val;
            v[0] += val;
        }
    }
    block_partials<1>(v, sm, part, 0);
}

__global__ __launch_bounds__(BLOCK) void k_apply(Dims d, Bc bc, const double *__restrict__ bx,
                                                 const double *__restrict__ by,
                                                 const double *__restrict__ bz,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ sg,
                                                 double *__restrict__ y, double ih2)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny)
        return;
    const Nb n = neighbours(d, bc, i, j, k);
    const Links<double> L = links(n, bx, by, bz);
    double v = ih2 * flux_sum(n, L, x);
    if (sg)
        v -= sg[n.c] * x[n.c];
    y[n.c] = v;
}

// u_m = us_m - dt beta_m G_m p on open faces, 0 on wall faces and on closed
// links (beta = 0: the link flags multiply the velocity) (eq. fotm).
// u may alias us: each thread reads and writes only its own entries.  RHO:
// beta formed from the cell densities (as in k_dir_apply).
template <bool RHO>
__global__ __launch_bounds__(BLOCK) void k_project(Dims d, Bc bc, const double *__restrict__ bx,
                                                   const double *__restrict__ by,
                                                   const double *__restrict__ bz,
                                                   const double *__restrict__ rho,
                                                   const double *usx, const double *usy,
                                                   const double *usz, const double *__restrict__ p,
                                                   double dt_h, double *ux, double *uy, double *uz)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny)
        return;
    const Nb n = neighbours(d, bc, i, j, k);
    const double pc = p[n.c];
    double fx, fy, fz;
    if (RHO) {   // beta from the densities, as the density load stores it
        const double rc = rho[n.c];
        fx = 2.0 / (rho[n.xm] + rc);
        fy = 2.0 / (rho[n.ym] + rc);
        fz = 2.0 / (rho[n.zm] + rc);
    } else {
        fx = bx[n.c];
        fy = by[n.c];
        fz = bz[n.c];
    }
    const double vx = (n.wxl || fx == 0.0) ? 0.0 : usx[n.c] - dt_h * fx * (pc - p[n.xm]);
    const double vy = (n.wyl || fy == 0.0) ? 0.0 : usy[n.c] - dt_h * fy * (pc - p[n.ym]);
    const double vz = (n.wzl || fz == 0.0) ? 0.0 : usz[n.c] - dt_h * fz * (pc - p[n.zm]);
    ux[n.c] = vx;
    uy[n.c] = vy;
    uz[n.c] = vz;
}

// g_beta_m = G_m lambda * G_m p on non-wall faces, 0 on walls
__global__ __launch_bounds__(BLOCK) void k_adjoint_faces(Dims d, Bc bc, const double *__restrict__ lam,
                                                         const double *__restrict__ p, double ih2,
                                                         const double *__restrict__ bx,
                                                         const double *__restrict__ by,
                                                         const double *__restrict__ bz,
                                                         double *__restrict__ gx,
                                                         double *__restrict__ gy,
                                                         double *__restrict__ gz)
{
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny)
        return;
    const Nb n = neighbours(d, bc, i, j, k);
    const double lc = lam[n.c], pc = p[n.c];
    const bool cx = bx && bx[n.c] == 0.0, cy = by && by[n.c] == 0.0, cz = bz && bz[n.c] == 0.0;
    gx[n.c] = (n.wxl || cx) ? 0.0 : ih2 * (lc - lam[n.xm]) * (pc - p[n.xm]);
    gy[n.c] = (n.wyl || cy) ? 0.0 : ih2 * (lc - lam[n.ym]) * (pc - p[n.ym]);
    gz[n.c] = (n.wzl || cz) ? 0.0 : ih2 * (lc - lam[n.zm]) * (pc - p[n.zm]);
}

// Streaming copy, the reference for achievable HBM bandwidth: one 16-byte
// vector per thread (a grid of n/512 workgroups), loaded and stored with the
// non-temporal hint, since nothing copied is read again soon.  Measured
// against a grid-stride loop with four vectors per thread in flight, and
// against workgroups that each copy a contiguous run of 2, 4 or 8 vectors
// per thread, this form is the fastest on MI355X (6.6 TB/s read + write on
// 1 GiB buffers).
__global__ __launch_bounds__(256) void k_copy(const double *__restrict__ src,
                                              double *__restrict__ dst, size_t n)
{
    using D2 = double __attribute__((ext_vector_type(2)));
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n / 2) {
        const D2 v = __builtin_nontemporal_load(reinterpret_cast<const D2 *>(src) + i);
        __builtin_nontemporal_store(v, reinterpret_cast<D2 *>(dst) + i);
    }
    if ((n & 1) && i == 0)
        dst[n - 1] = src[n - 1];
}

__global__ void k_copy_unaligned(const double *__restrict__ src, double *__restrict__ dst, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_fill(double *__restrict__ x, size_t n, double v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// ---------------------------------------------------------------------------
// outer-loop kernels (FP64) and reductions
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(BLOCK) void k_sum(Dims d, const double *__restrict__ x,
                                               const unsigned char *__restrict__ act, double *part)
{
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const size_t c = ((size_t)k * d.ny + j) * d.nx + i;
            if (!act || act[c])
                v[0] += x[c];
        }
    }
    block_partials<1>(v, sm, part, 0);
}

// Fixed-order sum of the partials (each thread a strided run, then the
// wave's lanes by butterfly shuffles, then the waves' sums in order), and the
// scalar update of `op`.  One barrier: the kernel is launched once or more
// per outer iteration and sits on the iteration's critical path.
constexpr int FIN_THREADS = 1024;
// host (may be null): pinned host memory that also receives the whole scalar
// array once the operation is done, written by the kernel itself so that the
// outer loop reads an iteration's scalars without a separate copy; then
// host[S_NSLOTS] = ticket, after the values (the host polls it)
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const double *__restrict__ part,
                                                          size_t pstride, int nparts, int op,
                                                          int slot, double ncells, int first,
                                                          double *scal, double *host,
                                                          double ticket)
{
    __shared__ double sm[2][FIN_THREADS / 64];
    const bool two = op == OP_INIT || op == OP_ALPHA;
    const int t = threadIdx.x;
    // four loads in flight per accumulation step (the sum order stays fixed)
    double a0 = 0.0, a1 = 0.0;
    int i = t;
    for (; i + 3 * FIN_THREADS < nparts; i += 4 * FIN_THREADS) {
        const double *p0 = part + i;
        a0 += (p0[0] + p0[FIN_THREADS]) + (p0[2 * FIN_THREADS] + p0[3 * FIN_THREADS]);
        if (two) {
            const double *p1 = part + pstride + i;
            a1 += (p1[0] + p1[FIN_THREADS]) + (p1[2 * FIN_THREADS] + p1[3 * FIN_THREADS]);
        }
    }
    for (; i < nparts; i += FIN_THREADS) {
        a0 += part[i];
        if (two)
            a1 += part[pstride + i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
    }
    if ((t & 63) == 0) {
        sm[0][t >> 6] = a0;
        sm[1][t >> 6] = a1;
    }
    __syncthreads();
    if (t != 0)
        return;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int w = 0; w < FIN_THREADS / 64; ++w) {
        s0 += sm[0][w];
        s1 += sm[1][w];
    }
    double rms;
    switch (op) {
    case OP_STORE:
        scal[slot] = s0;
        break;
    case OP_MEAN:
        scal[slot] = s0 / ncells;
        break;
    case OP_INIT:
        scal[S_RR] = s0;
        scal[S_BB] = s1;
        rms = sqrt(s0 / ncells);
        if (!(rms > 0.0) || !(rms < INFINITY))
            rms = 1.0;
        scal[S_USED] = rms;
        scal[S_NEXT] = rms;
        break;
    case OP_RZ:
    case OP_RZ_T: {
        // flexible CG: beta = (r_k . z_k - r_k . z_{k-1}) / (r_{k-1} . z_{k-1});
        // the stored direction is in units of the V-cycle scale, so its
        // recurrence coefficient is beta s_{k-1} / s_k.  OP_RZ_T: the partials
        // are of r / s_k, the right-hand side the V-cycle was given
        const double rz = (op == OP_RZ_T ? scal[S_USED] * scal[S_USED] : scal[S_USED]) * s0;
        scal[S_BETA] =
            first ? 0.0 : (rz - scal[S_RZOLD]) / scal[S_RZ] * (scal[S_DS] / scal[S_USED]);
        scal[S_RZ] = rz;
        break;
    }
    case OP_ALPHA:
        // s0 = D . A D with the true direction s_k D: alpha = rz / (s_k^2 s0);
        // the slot holds alpha s_k, the coefficient of D and of q = A D.
        // s1 = D_old . A D: since alpha_k (D_k . A D_k) = r_k . z_k and
        // D_k - z_k = beta_k D_{k-1}, the next residual against this z is
        // r_{k+1} . z_k = alpha_k beta_k (D_{k-1} . A D_k), in stored units
        // alpha s_k * gamma * s_k s1 / s_k (zero on the first iteration, whose
        // gamma is 0 and whose direction pass sums no s1)
        scal[S_DQ] = s0;
        scal[S_APREV] = scal[S_ALPHA];
        scal[S_ALPHA] = scal[S_RZ] / (scal[S_USED] * s0);
        scal[S_DS] = scal[S_USED];
        scal[S_RZOLD] = scal[S_ALPHA] * scal[S_BETA] * scal[S_USED] * s1;
        break;
    case OP_UPDATE:
        scal[S_RR] = s0;
        scal[S_USED] = scal[S_NEXT];
        rms = sqrt(s0 / ncells);
        scal[S_NEXT] = (rms > 0.0 && rms < INFINITY) ? rms : 1.0;
        break;
    case OP_DC:
        scal[S_RR] = s0;
        scal[S_USED] = scal[S_NEXT];
        rms = sqrt(s0 / ncells);
        scal[S_NEXT] = (rms > 0.0 && rms < INFINITY) ? rms : 1.0;
        break;
    default:
        break;
    }
    if (host) {
        for (int q = 0; q < S_NSLOTS; ++q)
            host[q] = scal[q];
        __threadfence_system();   // the values before the ticket
        *(volatile double *)(host + S_NSLOTS) = ticket;
        __threadfence_system();   // visible to the host before the kernel completes
    }
}

// n doubles from device memory to pinned, coherent host memory (one
// workgroup): the scalars and small arrays the host reads back
__global__ __launch_bounds__(256) void k_publish(const double *__restrict__ src, double *host, int n,
                                                double ticket)
{
    for (int q = threadIdx.x; q < n; q += blockDim.x)
        host[q] = src[q];
    __threadfence_system();
    if (ticket != 0.0) {
        // host[n] = ticket once every thread's values are out (the host polls it)
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence_system();
            *(volatile double *)(host + n) = ticket;
            __threadfence_system();
        }
    }
}

// r = (b - mean b) - A x; partials ||r||^2, ||b - mean b||^2 and the sum of
// x over the active cells (the gauge's mean, at no extra pass).
// ZEROX: x is set to zero (cold start) and A x is skipped.
template <bool ZEROX>
__global__ __launch_bounds__(BLOCK) void k_residual(Dims d, Bc bc, const double *__restrict__ bx,
                                                    const double *__restrict__ by,
                                                    const double *__restrict__ bz,
                                                    const double *__restrict__ b,
                                                    const double *__restrict__ scal, double *x,
                                                    const double *__restrict__ sg,
                                                    const unsigned char *__restrict__ act,
                                                    double *__restrict__ r64, double ih2,
                                                    double *part, size_t pstride)
{
    __shared__ double sm[3][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[3] = {0.0, 0.0, 0.0};
    if (i < d.nx && j < d.ny) {
        const double mean = scal[S_MEAN];
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const Nb n = neighbours(d, bc, i, j, k);
            // the right-hand side of an excluded cell is not part of the system
            const bool on = !act || act[n.c];
            const double bm = on ? b[n.c] - mean : 0.0;
            double ax = 0.0;
            if (ZEROX) {
                x[n.c] = 0.0;
            } else {
                const Links<double> L = links(n, bx, by, bz);
                ax = ih2 * flux_sum(n, L, x);
                if (sg)
                    ax -= sg[n.c] * x[n.c];
                if (on)
                    v[2] += x[n.c];
            }
            const double r = bm - ax;
            r64[n.c] = r;
            v[0] += r * r;
            v[1] += bm * bm;
        }
    }
    block_partials<3>(v, sm, part, pstride);
}

// k_residual (x given, the same three partial sums) for grids with even nx and ny and 16-byte aligned
// arrays: each thread owns a 2 x 2 block of cells and walks RZ planes with the
// column's planes below and at the current one carried in registers, as in
// k_dir_apply2; the same per-cell arithmetic as the one-cell kernel.  RHO: the
// link coefficients are formed from the cell densities by the expression the
// density load stores (same bits), reading 8 bytes per cell instead of 24.
template <bool RHO>
__global__ __launch_bounds__(BLOCK) void k_residual2(Dims d, Bc bc, const double *__restrict__ bx,
                                                     const double *__restrict__ by,
                                                     const double *__restrict__ bz,
                                                     const double *__restrict__ rho,
                                                     const double *__restrict__ b,
                                                     const double *__restrict__ scal,
                                                     const double *__restrict__ x,
                                                     const double *__restrict__ sg,
                                                     const unsigned char *__restrict__ act,
                                                     double *__restrict__ r64, double ih2,
                                                     double *part, size_t pstride)
{
    using F2 = double __attribute__((ext_vector_type(2)));
    __shared__ double sm[3][BLOCK / 64];
    unsigned gbx, gby, gbz;
    xcd_groups(gbx, gby, gbz);
    const int x0 = 2 * (int)(gbx * BX + threadIdx.x);
    const int j0 = 2 * (int)(gby * BY + threadIdx.y), j1 = j0 + 1;
    double v[3] = {0.0, 0.0, 0.0};
    if (x0 < d.nx && j0 < d.ny) {
        const double mean = scal[S_MEAN];
        const size_t sy = (size_t)d.nx, sz = (size_t)d.nx * d.ny;
        const int xm = (x0 == 0) ? d.nx - 1 : x0 - 1;
        const int xp = (x0 + 2 == d.nx) ? 0 : x0 + 2;
        const int jm = (j0 == 0) ? d.ny - 1 : j0 - 1;
        const int jp = (j1 + 1 == d.ny) ? 0 : j1 + 1;
        const bool wxl = bc.x && x0 == 0, wxh = bc.x && x0 + 2 == d.nx;
        const bool wyl = bc.y && j0 == 0, wyh = bc.y && j1 == d.ny - 1;
        const size_t o0 = (size_t)j0 * sy + x0, o1 = (size_t)j1 * sy + x0;
        const size_t om = (size_t)jm * sy + x0, op = (size_t)jp * sy + x0;
        const size_t m0 = (size_t)j0 * sy + xm, m1 = (size_t)j1 * sy + xm;
        const size_t p0 = (size_t)j0 * sy + xp, p1 = (size_t)j1 * sy + xp;
        auto ld2d = [](const double *p, size_t c) -> F2 {
            return *reinterpret_cast<const F2 *>(p + c);
        };
        auto quad = [&](const double *p, size_t pl, double (&o)[4]) {
            const F2 a = ld2d(p, pl + o0), c = ld2d(p, pl + o1);
            o[0] = a.x;
            o[1] = a.y;
            o[2] = c.x;
            o[3] = c.y;
        };
        // cells 0: (x0, j0), 1: (x0 + 1, j0), 2: (x0, j1), 3: (x0 + 1, j1)
        const int k0 = (int)gbz * RZ;
        const int ke = min(d.nz, k0 + RZ);
        const size_t pm0 = (size_t)(k0 == 0 ? d.nz - 1 : k0 - 1) * sz;
        double Xm[4], Xc[4], ZL[4], Rc[4];
        quad(x, pm0, Xm);
        quad(x, (size_t)k0 * sz, Xc);
        if (RHO) {
            double Rm[4];
            quad(rho, pm0, Rm);
            quad(rho, (size_t)k0 * sz, Rc);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                ZL[c] = 2.0 / (Rm[c] + Rc[c]);
        } else {
            quad(bz, (size_t)k0 * sz, ZL);
        }
        for (int k = k0; k < ke; ++k) {
            const size_t pl = (size_t)k * sz;
            const size_t pp = (size_t)(k == d.nz - 1 ? 0 : k + 1) * sz;
            double Xp[4], zh[4], bb[4], Rp[4];
            quad(x, pp, Xp);
            quad(b, pl, bb);
            const double xm0 = x[pl + m0], xp0 = x[pl + p0];
            const double xm1 = x[pl + m1], xp1 = x[pl + p1];
            const F2 xym = ld2d(x, pl + om), xyp = ld2d(x, pl + op);
            // x faces per row (low, middle, high), y faces per column
            double fx[2][3], fy[2][3];
            if (RHO) {
                quad(rho, pp, Rp);
                const double rxm0 = rho[pl + m0], rxp0 = rho[pl + p0];
                const double rxm1 = rho[pl + m1], rxp1 = rho[pl + p1];
                const F2 rym = ld2d(rho, pl + om), ryp = ld2d(rho, pl + op);
                fx[0][0] = 2.0 / (rxm0 + Rc[0]);
                fx[0][1] = 2.0 / (Rc[0] + Rc[1]);
                fx[0][2] = 2.0 / (Rc[1] + rxp0);
                fx[1][0] = 2.0 / (rxm1 + Rc[2]);
                fx[1][1] = 2.0 / (Rc[2] + Rc[3]);
                fx[1][2] = 2.0 / (Rc[3] + rxp1);
                fy[0][0] = 2.0 / (rym.x + Rc[0]);
                fy[0][1] = 2.0 / (Rc[0] + Rc[2]);
                fy[0][2] = 2.0 / (Rc[2] + ryp.x);
                fy[1][0] = 2.0 / (rym.y + Rc[1]);
                fy[1][1] = 2.0 / (Rc[1] + Rc[3]);
                fy[1][2] = 2.0 / (Rc[3] + ryp.y);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    zh[c] = 2.0 / (Rc[c] + Rp[c]);
            } else {
                quad(bz, pp, zh);
                const F2 bx0 = ld2d(bx, pl + o0), bx1 = ld2d(bx, pl + o1);
                const F2 by0 = ld2d(by, pl + o0), by1 = ld2d(by, pl + o1);
                const F2 byp = ld2d(by, pl + op);
                fx[0][0] = bx0.x;
                fx[0][1] = bx0.y;
                fx[0][2] = bx[pl + p0];
                fx[1][0] = bx1.x;
                fx[1][1] = bx1.y;
                fx[1][2] = bx[pl + p1];
                fy[0][0] = by0.x;
                fy[0][1] = by1.x;
                fy[0][2] = byp.x;
                fy[1][0] = by0.y;
                fy[1][1] = by1.y;
                fy[1][2] = byp.y;
            }
            const bool wzl = bc.z && k == 0, wzh = bc.z && k == d.nz - 1;
            const double nxm[4] = {xm0, Xc[0], xm1, Xc[2]};
            const double nxp[4] = {Xc[1], xp0, Xc[3], xp1};
            const double nym[4] = {xym.x, xym.y, Xc[0], Xc[1]};
            const double nyp[4] = {Xc[2], Xc[3], xyp.x, xyp.y};
            double rr[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int cx = c & 1, ry = c >> 1;
                const size_t cell = pl + (ry ? o1 : o0) + cx;
                const double Lxl = (cx == 0 && wxl) ? 0.0 : fx[ry][cx];
                const double Lxh = (cx == 1 && wxh) ? 0.0 : fx[ry][cx + 1];
                const double Lyl = (ry == 0 && wyl) ? 0.0 : fy[cx][ry];
                const double Lyh = (ry == 1 && wyh) ? 0.0 : fy[cx][ry + 1];
                const double Lzl = wzl ? 0.0 : ZL[c];
                const double Lzh = wzh ? 0.0 : zh[c];
                const double xc = Xc[c];
                // the right-hand side of an excluded cell is not part of the system
                const bool on = !act || act[cell];
                const double bm = on ? bb[c] - mean : 0.0;
                const double f = Lxh * (nxp[c] - xc) - Lxl * (xc - nxm[c]) +
                                 Lyh * (nyp[c] - xc) - Lyl * (xc - nym[c]) +
                                 Lzh * (Xp[c] - xc) - Lzl * (xc - Xm[c]);
                double ax = ih2 * f;
                if (sg)
                    ax -= sg[cell] * xc;
                rr[c] = bm - ax;
                v[0] += rr[c] * rr[c];
                v[1] += bm * bm;
                if (on)
                    v[2] += xc;
            }
            *reinterpret_cast<F2 *>(r64 + pl + o0) = F2{rr[0], rr[1]};
            *reinterpret_cast<F2 *>(r64 + pl + o1) = F2{rr[2], rr[3]};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                Xm[c] = Xc[c];
                Xc[c] = Xp[c];
                ZL[c] = zh[c];
                if (RHO)
                    Rc[c] = Rp[c];
            }
        }
    }
    block_partials<3>(v, sm, part, pstride);
}

// defect-correction residual: rT = ((b - mean b) - A x) / scal[S_NEXT]; partial ||r||^2
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_residual_T(Dims d, Bc bc, const double *__restrict__ bx,
                                                      const double *__restrict__ by,
                                                      const double *__restrict__ bz,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ scal,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ sg,
                                                      const unsigned char *__restrict__ act,
                                                      T *__restrict__ rT, double ih2, double *part)
{
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const double mean = scal[S_MEAN];
        const double inv = 1.0 / scal[S_NEXT];
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const Nb n = neighbours(d, bc, i, j, k);
            const Links<double> L = links(n, bx, by, bz);
            double ax = ih2 * flux_sum(n, L, x);
            if (sg)
                ax -= sg[n.c] * x[n.c];
            const double bm = (act && !act[n.c]) ? 0.0 : b[n.c] - mean;
            const double r = bm - ax;
            rT[n.c] = static_cast<T>(r * inv);
            v[0] += r * r;
        }
    }
    block_partials<1>(v, sm, part, 0);
}

template <typename T>
__global__ void k_scale_T(size_t n, const double *__restrict__ r, T *__restrict__ rT,
                          const double *__restrict__ scal)
{
    const double inv = 1.0 / scal[S_USED];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        rT[i] = static_cast<T>(r[i] * inv);
}

// x += scal[S_USED] * e
template <typename T>
__global__ void k_axpy_T(size_t n, const T *__restrict__ e, double *__restrict__ x,
                         const double *__restrict__ scal)
{
    const double s = scal[S_USED];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] += s * static_cast<double>(e[i]);
}

// partial r . z (z in storage precision; the scale is applied when finalising)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_dot_rz(Dims d, const double *__restrict__ r,
                                                  const T *__restrict__ z, double *part)
{
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const size_t c = ((size_t)k * d.ny + j) * d.nx + i;
            v[0] += r[c] * static_cast<double>(z[c]);
        }
    }
    block_partials<1>(v, sm, part, 0);
}

// New search direction and its image in one pass.  The direction is kept in
// units of the V-cycle's scale s_k = scal[S_USED] (the preconditioned
// residual is s_k z), so its storage type needs no range of its own:
//   D_new = z + gamma D_old    (gamma = scal[S_BETA] = beta_k s_{k-1} / s_k, or
//                               0 on the first iteration, when D_old is not read)
//   q = A D_new,  partial D_new . q
// and the true direction is s_k D_new.  D_new is rounded to its storage type
// before q is formed, so q is the image of exactly the stored vector; it is
// recomputed at the in-plane neighbours from z and D_old by the same explicit
// fma (so the same bits), which is why D_new and D_old are different buffers.
// The second partial is D_old . q, from which the flexible coefficient's
// r_{k+1} . z_k follows without a pass over z_k (see OP_ALPHA).
// Each thread walks a column of RZ planes and carries the column's values of
// the planes below and above (D_new, and the low z-face coefficient) in
// registers.  The iterate's updates are applied here, where D_old is read
// anyway, two directions at a time: MODE == DIR_TWO adds a_{k-2} D_{k-2}
// (D_{k-2} is what dnew holds until this pass overwrites it, a_{k-2} =
// scal[S_APREV]) and then a_{k-1} D_old (a_{k-1} = scal[S_ALPHA]; this launch
// runs before the new coefficient is finalised); DIR_HOLD leaves x alone, so
// its direction waits for the next pass, and DIR_FIRST has no D_old.
// RHO: the link coefficients are formed from the cell densities,
// beta = 2 / (rho_low + rho_high), the expression the density load stores, so
// q has the same bits as with the stored coefficients while 8 bytes per cell
// are read instead of 24.
template <typename T, typename D, int MODE, bool RHO>
__global__ __launch_bounds__(BLOCK) void k_dir_apply(Dims d, Bc bc, const double *__restrict__ bx,
                                                     const double *__restrict__ by,
                                                     const double *__restrict__ bz,
                                                     const double *__restrict__ rho,
                                                     const T *__restrict__ z,
                                                     const D *__restrict__ dold,
                                                     D *__restrict__ dnew,
                                                     double *__restrict__ q,
                                                     double *__restrict__ x,
                                                     const double *__restrict__ sg,
                                                     const double *__restrict__ scal, double ih2,
                                                     double *part, size_t pstride)
{
    __shared__ double sm[2][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[2] = {0.0, 0.0};
    constexpr bool FIRST = MODE == DIR_FIRST;
    if (i < d.nx && j < d.ny) {
        const double gamma = FIRST ? 0.0 : scal[S_BETA];
        const double aold = FIRST ? 0.0 : scal[S_ALPHA];
        const double aprev = MODE == DIR_TWO ? scal[S_APREV] : 0.0;
        auto dv = [&](size_t c) -> double {
            const double t = static_cast<double>(z[c]);
            return static_cast<double>(
                static_cast<D>(FIRST ? t : __builtin_fma(gamma, static_cast<double>(dold[c]), t)));
        };
        const size_t sz = (size_t)d.nx * d.ny;
        const size_t col = (size_t)j * d.nx + i;
        // in-plane neighbour offsets (periodic wrap; wall links are masked below)
        const ptrdiff_t oxm = (i == 0) ? d.nx - 1 : -1;
        const ptrdiff_t oxp = (i == d.nx - 1) ? -(ptrdiff_t)(d.nx - 1) : 1;
        const ptrdiff_t oym = (j == 0) ? (ptrdiff_t)(d.ny - 1) * d.nx : -(ptrdiff_t)d.nx;
        const ptrdiff_t oyp = (j == d.ny - 1) ? -(ptrdiff_t)(d.ny - 1) * d.nx : (ptrdiff_t)d.nx;
        const bool wxl = bc.x && i == 0, wxh = bc.x && i == d.nx - 1;
        const bool wyl = bc.y && j == 0, wyh = bc.y && j == d.ny - 1;
        const int k0 = blockIdx.z * RZ;
        const int ke = min(d.nz, k0 + RZ);
        const size_t cm0 = col + (size_t)(k0 == 0 ? d.nz - 1 : k0 - 1) * sz;
        double dm = dv(cm0), dc = dv(col + (size_t)k0 * sz);
        double rc = 0.0, zl;
        if (RHO) {
            rc = rho[col + (size_t)k0 * sz];
            zl = 2.0 / (rho[cm0] + rc);
        } else {
            zl = bz[col + (size_t)k0 * sz];
        }
        for (int k = k0; k < ke; ++k) {
            const size_t c = col + (size_t)k * sz;
            const size_t cp = col + (size_t)(k == d.nz - 1 ? 0 : k + 1) * sz;
            const double dp = dv(cp);
            double lxl, lxh, lyl, lyh, lzh;
            if (RHO) {
                const double rp = rho[cp];
                lxl = 2.0 / (rho[c + oxm] + rc);
                lxh = 2.0 / (rc + rho[c + oxp]);
                lyl = 2.0 / (rho[c + oym] + rc);
                lyh = 2.0 / (rc + rho[c + oyp]);
                lzh = 2.0 / (rc + rp);
                rc = rp;
            } else {
                lxl = bx[c];
                lxh = bx[c + oxp];
                lyl = by[c];
                lyh = by[c + oyp];
                lzh = bz[cp];
            }
            const double Lxl = wxl ? 0.0 : lxl, Lxh = wxh ? 0.0 : lxh;
            const double Lyl = wyl ? 0.0 : lyl, Lyh = wyh ? 0.0 : lyh;
            const double Lzl = (bc.z && k == 0) ? 0.0 : zl;
            const double Lzh = (bc.z && k == d.nz - 1) ? 0.0 : lzh;
            const double f = Lxh * (dv(c + oxp) - dc) - Lxl * (dc - dv(c + oxm)) +
                             Lyh * (dv(c + oyp) - dc) - Lyl * (dc - dv(c + oym)) +
                             Lzh * (dp - dc) - Lzl * (dc - dm);
            double qq = ih2 * f;
            if (sg)
                qq -= sg[c] * dc;
            if (!FIRST) {
                const double dold_c = static_cast<double>(dold[c]);
                if (MODE == DIR_TWO)
                    x[c] = (x[c] + aprev * static_cast<double>(dnew[c])) + aold * dold_c;
                v[1] += dold_c * qq;
            }
            dnew[c] = static_cast<D>(dc);
            q[c] = qq;
            v[0] += dc * qq;
            zl = lzh;
            dm = dc;
            dc = dp;
        }
    }
    block_partials<2>(v, sm, part, pstride);
}

// k_dir_apply for grids with even nx and ny (and a 16-byte aligned iterate):
// each thread owns a 2 x 2 block of cells, an x-pair in two rows, so a
// workgroup covers 128 x 8 cells of each plane.  Workgroups are dispatched to
// the XCDs in turn, so the halo rows and lines a workgroup shares with its
// neighbours are fetched again by another XCD's L2; per cell there are half as
// many of them here.  The faces between the block's cells are formed once.
// Same arithmetic per cell as k_dir_apply (same order of terms), and the same
// iterate updates (MODE).
template <typename T, typename D, int MODE, bool RHO>
__global__ __launch_bounds__(BLOCK) void k_dir_apply2(Dims d, Bc bc, const double *__restrict__ bx,
                                                      const double *__restrict__ by,
                                                      const double *__restrict__ bz,
                                                      const double *__restrict__ rho,
                                                      const T *__restrict__ z,
                                                      const D *__restrict__ dold,
                                                      D *__restrict__ dnew,
                                                      double *__restrict__ q,
                                                      double *__restrict__ x,
                                                      const double *__restrict__ sg,
                                                      const double *__restrict__ scal, double ih2,
                                                      double *part, size_t pstride)
{
    using T2 = typename Vec2<T>::type;
    using D2 = typename Vec2<D>::type;
    using F2 = double __attribute__((ext_vector_type(2)));
    __shared__ double sm[2][BLOCK / 64];
    unsigned gbx, gby, gbz;
    xcd_groups(gbx, gby, gbz);
    const int x0 = 2 * (int)(gbx * BX + threadIdx.x);
    const int j0 = 2 * (int)(gby * BY + threadIdx.y), j1 = j0 + 1;
    double v[2] = {0.0, 0.0};
    constexpr bool FIRST = MODE == DIR_FIRST;
    if (x0 < d.nx && j0 < d.ny) {
        const double gamma = FIRST ? 0.0 : scal[S_BETA];
        const double aold = FIRST ? 0.0 : scal[S_ALPHA];
        const double aprev = MODE == DIR_TWO ? scal[S_APREV] : 0.0;
        const size_t sy = (size_t)d.nx, sz = (size_t)d.nx * d.ny;
        const int xm = (x0 == 0) ? d.nx - 1 : x0 - 1;
        const int xp = (x0 + 2 == d.nx) ? 0 : x0 + 2;
        const int jm = (j0 == 0) ? d.ny - 1 : j0 - 1;
        const int jp = (j1 + 1 == d.ny) ? 0 : j1 + 1;
        const bool wxl = bc.x && x0 == 0, wxh = bc.x && x0 + 2 == d.nx;
        const bool wyl = bc.y && j0 == 0, wyh = bc.y && j1 == d.ny - 1;
        // in-plane offsets: the pair in rows j0 and j1, the pair in the rows
        // beyond them, the cells beyond the pair in rows j0 and j1
        const size_t o0 = (size_t)j0 * sy + x0, o1 = (size_t)j1 * sy + x0;
        const size_t om = (size_t)jm * sy + x0, op = (size_t)jp * sy + x0;
        const size_t m0 = (size_t)j0 * sy + xm, m1 = (size_t)j1 * sy + xm;
        const size_t p0 = (size_t)j0 * sy + xp, p1 = (size_t)j1 * sy + xp;
        auto dcast = [&](double t, double o) -> double {
            return static_cast<double>(static_cast<D>(FIRST ? t : __builtin_fma(gamma, o, t)));
        };
        auto dv1 = [&](size_t c) -> double {
            return dcast(static_cast<double>(z[c]), FIRST ? 0.0 : static_cast<double>(dold[c]));
        };
        // the direction at a pair, and D_old there
        auto dv2 = [&](size_t c, double &a, double &b, double &oa, double &ob) {
            const T2 t = *reinterpret_cast<const T2 *>(z + c);
            oa = ob = 0.0;
            if (!FIRST) {
                const D2 o = *reinterpret_cast<const D2 *>(dold + c);
                oa = static_cast<double>(o.x);
                ob = static_cast<double>(o.y);
            }
            a = dcast(static_cast<double>(t.x), oa);
            b = dcast(static_cast<double>(t.y), ob);
        };
        auto ld2d = [](const double *p, size_t c) -> F2 {
            return *reinterpret_cast<const F2 *>(p + c);
        };
        // cells 0: (x0, j0), 1: (x0 + 1, j0), 2: (x0, j1), 3: (x0 + 1, j1)
        const int k0 = (int)gbz * RZ;
        const int ke = min(d.nz, k0 + RZ);
        const size_t pm = (size_t)(k0 == 0 ? d.nz - 1 : k0 - 1) * sz, pc0 = (size_t)k0 * sz;
        double Dm[4], Dc[4], Oc[4], ZL[4], Rc[4], t0, t1;
        dv2(pm + o0, Dm[0], Dm[1], t0, t1);
        dv2(pm + o1, Dm[2], Dm[3], t0, t1);
        dv2(pc0 + o0, Dc[0], Dc[1], Oc[0], Oc[1]);
        dv2(pc0 + o1, Dc[2], Dc[3], Oc[2], Oc[3]);
        if (RHO) {
            const F2 a0 = ld2d(rho, pm + o0), a1 = ld2d(rho, pm + o1);
            const F2 c0 = ld2d(rho, pc0 + o0), c1 = ld2d(rho, pc0 + o1);
            Rc[0] = c0.x;
            Rc[1] = c0.y;
            Rc[2] = c1.x;
            Rc[3] = c1.y;
            ZL[0] = 2.0 / (a0.x + Rc[0]);
            ZL[1] = 2.0 / (a0.y + Rc[1]);
            ZL[2] = 2.0 / (a1.x + Rc[2]);
            ZL[3] = 2.0 / (a1.y + Rc[3]);
        } else {
            const F2 c0 = ld2d(bz, pc0 + o0), c1 = ld2d(bz, pc0 + o1);
            ZL[0] = c0.x;
            ZL[1] = c0.y;
            ZL[2] = c1.x;
            ZL[3] = c1.y;
        }
        for (int k = k0; k < ke; ++k) {
            const size_t pl = (size_t)k * sz;
            const size_t pp = (size_t)(k == d.nz - 1 ? 0 : k + 1) * sz;
            double Dp[4], Op[4];
            dv2(pp + o0, Dp[0], Dp[1], Op[0], Op[1]);
            dv2(pp + o1, Dp[2], Dp[3], Op[2], Op[3]);
            // the direction beyond the block in this plane
            const double dxm0 = dv1(pl + m0), dxp0 = dv1(pl + p0);
            const double dxm1 = dv1(pl + m1), dxp1 = dv1(pl + p1);
            double dym0, dym1, dyp0, dyp1;
            dv2(pl + om, dym0, dym1, t0, t1);
            dv2(pl + op, dyp0, dyp1, t0, t1);
            // link coefficients: x faces per row (low, middle, high), y faces
            // per column (low, middle, high), the high z faces
            double fx[2][3], fy[2][3], zh[4], Rp[4];
            if (RHO) {
                const F2 a0 = ld2d(rho, pp + o0), a1 = ld2d(rho, pp + o1);
                Rp[0] = a0.x;
                Rp[1] = a0.y;
                Rp[2] = a1.x;
                Rp[3] = a1.y;
                const double rxm0 = rho[pl + m0], rxp0 = rho[pl + p0];
                const double rxm1 = rho[pl + m1], rxp1 = rho[pl + p1];
                const F2 rym = ld2d(rho, pl + om), ryp = ld2d(rho, pl + op);
                fx[0][0] = 2.0 / (rxm0 + Rc[0]);
                fx[0][1] = 2.0 / (Rc[0] + Rc[1]);
                fx[0][2] = 2.0 / (Rc[1] + rxp0);
                fx[1][0] = 2.0 / (rxm1 + Rc[2]);
                fx[1][1] = 2.0 / (Rc[2] + Rc[3]);
                fx[1][2] = 2.0 / (Rc[3] + rxp1);
                fy[0][0] = 2.0 / (rym.x + Rc[0]);
                fy[0][1] = 2.0 / (Rc[0] + Rc[2]);
                fy[0][2] = 2.0 / (Rc[2] + ryp.x);
                fy[1][0] = 2.0 / (rym.y + Rc[1]);
                fy[1][1] = 2.0 / (Rc[1] + Rc[3]);
                fy[1][2] = 2.0 / (Rc[3] + ryp.y);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    zh[c] = 2.0 / (Rc[c] + Rp[c]);
            } else {
                const F2 bx0 = ld2d(bx, pl + o0), bx1 = ld2d(bx, pl + o1);
                const F2 by0 = ld2d(by, pl + o0), by1 = ld2d(by, pl + o1);
                const F2 byp = ld2d(by, pl + op);
                const F2 bz0 = ld2d(bz, pp + o0), bz1 = ld2d(bz, pp + o1);
                fx[0][0] = bx0.x;
                fx[0][1] = bx0.y;
                fx[0][2] = bx[pl + p0];
                fx[1][0] = bx1.x;
                fx[1][1] = bx1.y;
                fx[1][2] = bx[pl + p1];
                fy[0][0] = by0.x;
                fy[0][1] = by1.x;
                fy[0][2] = byp.x;
                fy[1][0] = by0.y;
                fy[1][1] = by1.y;
                fy[1][2] = byp.y;
                zh[0] = bz0.x;
                zh[1] = bz0.y;
                zh[2] = bz1.x;
                zh[3] = bz1.y;
            }
            const bool wzl = bc.z && k == 0, wzh = bc.z && k == d.nz - 1;
            // per cell: x column cx, row ry; neighbours in x and y
            const double nxm[4] = {dxm0, Dc[0], dxm1, Dc[2]};
            const double nxp[4] = {Dc[1], dxp0, Dc[3], dxp1};
            const double nym[4] = {dym0, dym1, Dc[0], Dc[1]};
            const double nyp[4] = {Dc[2], Dc[3], dyp0, dyp1};
            double qq[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int cx = c & 1, ry = c >> 1;
                const double Lxl = (cx == 0 && wxl) ? 0.0 : fx[ry][cx];
                const double Lxh = (cx == 1 && wxh) ? 0.0 : fx[ry][cx + 1];
                const double Lyl = (ry == 0 && wyl) ? 0.0 : fy[cx][ry];
                const double Lyh = (ry == 1 && wyh) ? 0.0 : fy[cx][ry + 1];
                const double Lzl = wzl ? 0.0 : ZL[c];
                const double Lzh = wzh ? 0.0 : zh[c];
                const double dc = Dc[c];
                const double f = Lxh * (nxp[c] - dc) - Lxl * (dc - nxm[c]) +
                                 Lyh * (nyp[c] - dc) - Lyl * (dc - nym[c]) +
                                 Lzh * (Dp[c] - dc) - Lzl * (dc - Dm[c]);
                qq[c] = ih2 * f;
                if (sg)
                    qq[c] -= sg[pl + (ry ? o1 : o0) + cx] * dc;
            }
            if (MODE == DIR_TWO) {
                // D_{k-2} is what dnew holds until the stores below
                const D2 ea = *reinterpret_cast<const D2 *>(dnew + pl + o0);
                const D2 eb = *reinterpret_cast<const D2 *>(dnew + pl + o1);
                F2 *xa = reinterpret_cast<F2 *>(x + pl + o0);
                F2 *xb = reinterpret_cast<F2 *>(x + pl + o1);
                F2 va = *xa, vb = *xb;
                va.x = (va.x + aprev * static_cast<double>(ea.x)) + aold * Oc[0];
                va.y = (va.y + aprev * static_cast<double>(ea.y)) + aold * Oc[1];
                vb.x = (vb.x + aprev * static_cast<double>(eb.x)) + aold * Oc[2];
                vb.y = (vb.y + aprev * static_cast<double>(eb.y)) + aold * Oc[3];
                *xa = va;
                *xb = vb;
            }
            *reinterpret_cast<D2 *>(dnew + pl + o0) = D2{static_cast<D>(Dc[0]), static_cast<D>(Dc[1])};
            *reinterpret_cast<D2 *>(dnew + pl + o1) = D2{static_cast<D>(Dc[2]), static_cast<D>(Dc[3])};
            *reinterpret_cast<F2 *>(q + pl + o0) = F2{qq[0], qq[1]};
            *reinterpret_cast<F2 *>(q + pl + o1) = F2{qq[2], qq[3]};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                v[0] += Dc[c] * qq[c];
                if (!FIRST)
                    v[1] += Oc[c] * qq[c];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ZL[c] = zh[c];
                Dm[c] = Dc[c];
                Dc[c] = Dp[c];
                Oc[c] = Op[c];
                if (RHO)
                    Rc[c] = Rp[c];
            }
        }
    }
    block_partials<2>(v, sm, part, pstride);
}

// r -= a q (a = scal[S_ALPHA]); rT = r / scal[S_NEXT]; partial ||r||^2.
// The iterate takes the matching x += a D in a later direction pass (two
// directions at a time), or in k_axpy_dir after the last iteration.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_pcg_update(Dims d, const double *__restrict__ q,
                                                      double *__restrict__ r, T *__restrict__ rT,
                                                      const double *__restrict__ scal,
                                                      double *part)
{
    __shared__ double sm[1][BLOCK / 64];
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    double v[1] = {0.0};
    if (i < d.nx && j < d.ny) {
        const double alpha = scal[S_ALPHA];
        const double inv = 1.0 / scal[S_NEXT];
        const int ke = min(d.nz, ((int)blockIdx.z + 1) * RZ);
        for (int k = blockIdx.z * RZ; k < ke; ++k) {
            const size_t c = ((size_t)k * d.ny + j) * d.nx + i;
            const double rn = r[c] - alpha * q[c];
            r[c] = rn;
            rT[c] = static_cast<T>(rn * inv);
            v[0] += rn * rn;
        }
    }
    block_partials<1>(v, sm, part, 0);
}

// x += scal[S_ALPHA] * D (after x += scal[S_APREV] * D_prev when given): the
// updates of the iterate still pending after the last iteration
template <typename D>
__global__ void k_axpy_dir(size_t n, const D *__restrict__ dv, const D *__restrict__ dv_prev,
                           double *__restrict__ x, const double *__restrict__ scal)
{
    const double a = scal[S_ALPHA];
    const double ap = dv_prev ? scal[S_APREV] : 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        double v = x[i];
        if (dv_prev)
            v += ap * static_cast<double>(dv_prev[i]);
        x[i] = v + a * static_cast<double>(dv[i]);
    }
}

// k_axpy_dir on four cells per thread and step, as 16-byte vectors (n
// divisible by 4 and aligned arrays): the same arithmetic per cell
template <typename D>
__global__ void k_axpy_dir4(size_t n4, const D *__restrict__ dv, const D *__restrict__ dv_prev,
                            double *__restrict__ x, const double *__restrict__ scal)
{
    using F2 = double __attribute__((ext_vector_type(2)));
    using D4 = D __attribute__((ext_vector_type(4)));
    const double a = scal[S_ALPHA];
    const double ap = dv_prev ? scal[S_APREV] : 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x) {
        const F2 x0 = reinterpret_cast<const F2 *>(x)[2 * i];
        const F2 x1 = reinterpret_cast<const F2 *>(x)[2 * i + 1];
        const D4 d = reinterpret_cast<const D4 *>(dv)[i];
        double v[4] = {x0.x, x0.y, x1.x, x1.y};
        if (dv_prev) {
            const D4 dp = reinterpret_cast<const D4 *>(dv_prev)[i];
            v[0] += ap * static_cast<double>(dp.x);
            v[1] += ap * static_cast<double>(dp.y);
            v[2] += ap * static_cast<double>(dp.z);
            v[3] += ap * static_cast<double>(dp.w);
        }
        v[0] = v[0] + a * static_cast<double>(d.x);
        v[1] = v[1] + a * static_cast<double>(d.y);
        v[2] = v[2] + a * static_cast<double>(d.z);
        v[3] = v[3] + a * static_cast<double>(d.w);
        reinterpret_cast<F2 *>(x)[2 * i] = F2{v[0], v[1]};
        reinterpret_cast<F2 *>(x)[2 * i + 1] = F2{v[2], v[3]};
    }
}

__global__ void k_sub_mean(size_t n, double *__restrict__ x, const double *__restrict__ scal, int slot,
                           const unsigned char *__restrict__ act)
{
    const double m = slot >= 0 ? scal[slot] : 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = (act && !act[i]) ? 0.0 : x[i] - m;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline dim3 flat_grid(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > 16384)
        b = 16384;
    if (b == 0)
        b = 1;
    return dim3((unsigned)b);
}

static const dim3 kBlock(BX, BY, 1);

template <typename T>
void launch_rbgs(Dims d, Bc bc, const T *bx, const T *by, const T *bz, const T *r, T *e,
                 const T *sg, double h2, double omega, int colour, bool zero, bool self_zero,
                 hipStream_t s)
{
    using C = typename Acc<T>::type;
    if (zero)
        hipLaunchKernelGGL((k_rbgs<T, true>), colour_grid(d), kBlock, 0, s, d, bc, bx, by, bz, r, e,
                           sg, (C)h2, (C)omega, colour, 1);
    else
        hipLaunchKernelGGL((k_rbgs<T, false>), colour_grid(d), kBlock, 0, s, d, bc, bx, by, bz, r,
                           e, sg, (C)h2, (C)omega, colour, self_zero ? 1 : 0);
}

template <typename T>
void launch_resid_restrict(Dims fd, Bc bc, const T *bx, const T *by, const T *bz, const T *e,
                           const T *r, const T *sg, T *rH, double ih2, hipStream_t s)
{
    using C = typename Acc<T>::type;
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    // coarse planes per thread: the longest walk (up to 4) that still leaves
    // at least 1024 workgroups, so the machine stays full
    dim3 g = cell_grid(cd);
    int kz = 1;
    while (kz < 4 && (size_t)g.x * g.y * ((cd.nz + 2 * kz - 1) / (2 * kz)) >= 1024)
        kz *= 2;
    g.z = (cd.nz + kz - 1) / kz;
    PP_LAUNCH((k_resid_restrict<T>), g, kBlock, 0, s, fd, bc, bx, by, bz, e, r, sg, rH,
              (C)ih2, kz);
}

template <typename T>
void launch_prolong(Dims fd, Bc bc, const T *eH, T *e, const unsigned *w, hipStream_t s)
{
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    PP_LAUNCH((k_prolong<T>), cell_grid(cd), kBlock, 0, s, fd, bc, eH, e, w);
}

void launch_prolong_weights(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                            unsigned *w, hipStream_t s)
{
    hipLaunchKernelGGL(k_prolong_weights, cell_grid(d), kBlock, 0, s, d, bc, bx, by, bz, w);
}

template <typename T>
void launch_tail(int nlev, const Dims *d, const double *h2, const void *const (*b)[3], void *const *e,
                 void *const *r, const void *const *sg, const unsigned *const *w, Bc bc,
                 int nu_pre, int nu_post, double omega, const double *pinv, int ncoarse,
                 bool warm, hipStream_t s)
{
    TailArgs<T> a;
    a.n = nlev;
    for (int l = 0; l < nlev; ++l) {
        a.d[l] = d[l];
        a.h2[l] = h2[l];
        for (int m = 0; m < 3; ++m)
            a.b[l][m] = (const T *)b[l][m];
        a.w[l] = w ? w[l] : nullptr;
        a.e[l] = (T *)e[l];
        a.r[l] = (T *)r[l];
        a.s[l] = (const T *)sg[l];
    }
    a.bc = bc;
    a.nu_pre = nu_pre;
    a.nu_post = nu_post;
    a.omega = omega;
    a.warm = warm ? 1 : 0;
    a.pinv = pinv;
    a.ncoarse = ncoarse;
    hipLaunchKernelGGL((k_tail_cycle<T>), dim3(1), dim3(TAIL_THREADS), 0, s, a);
}

template <typename T>
void launch_coarsest(int n, const double *pinv, const T *r, T *e, hipStream_t s)
{
    int threads = ((n + 63) / 64) * 64;
    if (threads > 1024)
        threads = 1024;
    hipLaunchKernelGGL((k_coarsest<T>), dim3(1), dim3(threads), 0, s, n, pinv, r, e);
}

template <typename T>
int launch_convert_scaled(size_t n, const double *src, double scale, double limit, T *dst,
                          double *part, int max_blocks, hipStream_t s)
{
    dim3 g = flat_grid(n);
    if ((int)g.x > max_blocks)
        g.x = max_blocks;                 // the loop strides over the rest
    hipLaunchKernelGGL((k_convert_scaled<T>), g, dim3(256), 0, s, n, src, scale, limit, dst, part);
    return (int)g.x;
}

template <typename T>
void launch_convert(size_t n, const double *src, T *dst, hipStream_t s)
{
    hipLaunchKernelGGL((k_convert<T>), flat_grid(n), dim3(256), 0, s, n, src, dst);
}

template <typename T>
void launch_to_double(size_t n, const T *src, double *dst, hipStream_t s)
{
    hipLaunchKernelGGL((k_to_double<T>), flat_grid(n), dim3(256), 0, s, n, src, dst);
}

void launch_coarsen_beta(Dims fd, Bc bc, const double *bx, const double *by, const double *bz,
                         double *hx, double *hy, double *hz, hipStream_t s)
{
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    hipLaunchKernelGGL(k_coarsen_beta, cell_grid(cd), kBlock, 0, s, fd, bc, bx, by, bz, hx, hy, hz);
}

void launch_zero_walls(Dims d, Bc bc, double *bx, double *by, double *bz, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_walls, cell_grid(d), kBlock, 0, s, d, bc, bx, by, bz);
}

template <typename T>
int launch_load_coeffs(Dims fd, Bc bc, const double *const src[3], double *const dst[3],
                       T *const dstT[3], double *const coarse[3], unsigned *w0, double *part,
                       hipStream_t s, T *const coarseT[3])
{
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const int kz = part ? RZ / 2 : 1;
    const dim3 g((cd.nx + BX - 1) / BX, (cd.ny + BY - 1) / BY, (cd.nz + kz - 1) / kz);
    T *ct[3] = {nullptr, nullptr, nullptr};
    if (coarseT)
        for (int m = 0; m < 3; ++m)
            ct[m] = coarseT[m];
    if (dstT[0])
        hipLaunchKernelGGL((k_load_coeffs<T, true>), g, kBlock, 0, s, fd, bc, src[0], src[1], src[2],
                           dst[0], dst[1], dst[2], dstT[0], dstT[1], dstT[2], coarse[0], coarse[1],
                           coarse[2], ct[0], ct[1], ct[2], w0, part, kz);
    else
        hipLaunchKernelGGL((k_load_coeffs<T, false>), g, kBlock, 0, s, fd, bc, src[0], src[1],
                           src[2], dst[0], dst[1], dst[2], dstT[0], dstT[1], dstT[2], coarse[0],
                           coarse[1], coarse[2], ct[0], ct[1], ct[2], w0, part, kz);
    return part ? (int)grid_blocks(g) : 0;
}

template <typename T>
int launch_load_density(Dims fd, Bc bc, const double *rho, double *const dst[3], T *const dstT[3],
                        double *const coarse[3], double *rcopy, unsigned *w0, double *part,
                        hipStream_t s)
{
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    const dim3 g((cd.nx + BX - 1) / BX, (cd.ny + BY - 1) / BY, (cd.nz + RZ / 2 - 1) / (RZ / 2));
    if (dstT[0])
        hipLaunchKernelGGL((k_load_density<T, true>), g, kBlock, 0, s, fd, bc, rho, dst[0], dst[1],
                           dst[2], dstT[0], dstT[1], dstT[2], coarse[0], coarse[1], coarse[2],
                           rcopy, w0, part);
    else
        hipLaunchKernelGGL((k_load_density<T, false>), g, kBlock, 0, s, fd, bc, rho, dst[0], dst[1],
                           dst[2], dstT[0], dstT[1], dstT[2], coarse[0], coarse[1], coarse[2],
                           rcopy, w0, part);
    return (int)grid_blocks(g);
}

void launch_check_rho(Dims d, const double *rho, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_rho, red_grid(d), kBlock, 0, s, d, rho, part);
}

void launch_check_beta(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                       bool allow_zero, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_beta, red_grid(d), kBlock, 0, s, d, bc, bx, by, bz,
                       allow_zero ? 1 : 0, part);
}

void launch_check_sigma(Dims d, const double *sg, double *part, size_t pstride, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_sigma, red_grid(d), kBlock, 0, s, d, sg, part, pstride);
}

void launch_active(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                   const double *sg, unsigned char *act, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_active, red_grid(d), kBlock, 0, s, d, bc, bx, by, bz, sg, act, part);
}

void launch_coarsen_sigma(Dims fd, const double *sg, double *sH, hipStream_t s)
{
    const Dims cd{fd.nx / 2, fd.ny / 2, fd.nz / 2};
    hipLaunchKernelGGL(k_coarsen_sigma, cell_grid(cd), kBlock, 0, s, fd, sg, sH);
}

void launch_mask(size_t n, double *x, const unsigned char *act, hipStream_t s)
{
    hipLaunchKernelGGL(k_mask, flat_grid(n), dim3(256), 0, s, n, x, act);
}

void launch_face_coeffs(Dims d, Bc bc, const double *rho, double *bx, double *by, double *bz,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_face_coeffs, cell_grid(d), kBlock, 0, s, d, bc, rho, bx, by, bz);
}

int launch_divergence_sum(Dims d, Bc bc, const double *ux, const double *uy, const double *uz,
                          double scale_over_h, double *out, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_divergence_sum, red_grid(d), kBlock, 0, s, d, bc, ux, uy, uz,
                       scale_over_h, out, part);
    return (int)grid_blocks(red_grid(d));
}

void launch_divergence(Dims d, Bc bc, const double *ux, const double *uy, const double *uz,
                       double scale_over_h, const double *bx, const double *by, const double *bz,
                       double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_divergence, cell_grid(d), kBlock, 0, s, d, bc, ux, uy, uz, scale_over_h,
                       bx, by, bz, out);
}

void launch_apply(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                  const double *x, const double *sg, double *y, double ih2, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply, cell_grid(d), kBlock, 0, s, d, bc, bx, by, bz, x, sg, y, ih2);
}

void launch_project(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                    const double *rho, const double *usx, const double *usy, const double *usz,
                    const double *p, double dt_over_h, double *ux, double *uy, double *uz,
                    hipStream_t s)
{
    if (rho)
        hipLaunchKernelGGL(k_project<true>, cell_grid(d), kBlock, 0, s, d, bc, bx, by, bz, rho, usx,
                           usy, usz, p, dt_over_h, ux, uy, uz);
    else
        hipLaunchKernelGGL(k_project<false>, cell_grid(d), kBlock, 0, s, d, bc, bx, by, bz, rho,
                           usx, usy, usz, p, dt_over_h, ux, uy, uz);
}

void launch_adjoint_faces(Dims d, Bc bc, const double *lam, const double *p, double ih2,
                          const double *bx, const double *by, const double *bz, double *gx,
                          double *gy, double *gz, hipStream_t s)
{
    hipLaunchKernelGGL(k_adjoint_faces, cell_grid(d), kBlock, 0, s, d, bc, lam, p, ih2, bx, by, bz,
                       gx, gy, gz);
}

void launch_copy(const double *src, double *dst, size_t n, hipStream_t s)
{
    // 16-byte accesses need 16-byte aligned pointers, otherwise the plain loop
    if (((uintptr_t)src | (uintptr_t)dst) & 15)
        hipLaunchKernelGGL(k_copy_unaligned, flat_grid(n), dim3(256), 0, s, src, dst, n);
    else
        hipLaunchKernelGGL(k_copy, dim3((unsigned)((n / 2 + 255) / 256) + 1), dim3(256), 0, s,
                           src, dst, n);
}

void launch_fill(double *x, size_t n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, flat_grid(n), dim3(256), 0, s, x, n, v);
}

void launch_sum(Dims d, const double *x, const unsigned char *act, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum, red_grid(d), kBlock, 0, s, d, x, act, part);
}

// up to four arrays of n doubles, one after the other into host
struct PublishSrc {
    const double *p[4];
};

__global__ __launch_bounds__(256) void k_publish_arrays(PublishSrc src, int narr, int n, double *host)
{
    for (int a = 0; a < narr; ++a)
        for (int q = threadIdx.x; q < n; q += blockDim.x)
            host[(size_t)a * n + q] = src.p[a][q];
    __threadfence_system();
}

void launch_publish_arrays(const double *const *src, int narr, int n, double *host, hipStream_t s)
{
    PublishSrc ps{{nullptr, nullptr, nullptr, nullptr}};
    for (int a = 0; a < narr && a < 4; ++a)
        ps.p[a] = src[a];
    hipLaunchKernelGGL(k_publish_arrays, dim3(1), dim3(256), 0, s, ps, narr < 4 ? narr : 4, n,
                       host);
}

void launch_publish(const double *src, double *host, int n, hipStream_t s, double ticket)
{
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, s, src, host, n, ticket);
}

void launch_finalize(const double *part, size_t pstride, int nparts, int op, int slot,
                     double ncells, int first, double *scal, hipStream_t s, double *host,
                     double ticket)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, s, part, pstride, nparts, op, slot,
                       ncells, first, scal, host, ticket);
}

int launch_residual(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                    const double *rho, const double *b, const double *scal, double *x, bool zero_x,
                    const double *sg, const unsigned char *act, double *r64, double ih2,
                    double *part, size_t pstride, hipStream_t s)
{
    const bool quad = !zero_x && d.nx % 2 == 0 && d.ny % 2 == 0 &&
                      (((uintptr_t)x | (uintptr_t)b | (uintptr_t)r64) & 15) == 0;
    if (quad) {
        const dim3 g((d.nx / 2 + BX - 1) / BX, (d.ny / 2 + BY - 1) / BY, (d.nz + RZ - 1) / RZ);
        if (residual_from_rho(d, rho, b, x, r64))
            hipLaunchKernelGGL(k_residual2<true>, g, kBlock, 0, s, d, bc, bx, by, bz, rho, b, scal,
                               x, sg, act, r64, ih2, part, pstride);
        else
            hipLaunchKernelGGL(k_residual2<false>, g, kBlock, 0, s, d, bc, bx, by, bz, nullptr, b,
                               scal, x, sg, act, r64, ih2, part, pstride);
        return (int)grid_blocks(g);
    }
    if (zero_x)
        hipLaunchKernelGGL(k_residual<true>, red_grid(d), kBlock, 0, s, d, bc, bx, by, bz, b, scal,
                           x, sg, act, r64, ih2, part, pstride);
    else
        hipLaunchKernelGGL(k_residual<false>, red_grid(d), kBlock, 0, s, d, bc, bx, by, bz, b,
                           scal, x, sg, act, r64, ih2, part, pstride);
    return (int)grid_blocks(red_grid(d));
}

template <typename T>
void launch_residual_T(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                       const double *b, const double *scal, const double *x, const double *sg,
                       const unsigned char *act, T *rT, double ih2, double *part, hipStream_t s)
{
    PP_LAUNCH((k_residual_T<T>), red_grid(d), kBlock, 0, s, d, bc, bx, by, bz, b, scal, x,
              sg, act, rT, ih2, part);
}

template <typename T>
void launch_scale_T(size_t n, const double *r, T *rT, const double *scal, hipStream_t s)
{
    hipLaunchKernelGGL((k_scale_T<T>), flat_grid(n), dim3(256), 0, s, n, r, rT, scal);
}

template <typename T>
void launch_axpy_T(size_t n, const T *e, double *x, const double *scal, hipStream_t s)
{
    hipLaunchKernelGGL((k_axpy_T<T>), flat_grid(n), dim3(256), 0, s, n, e, x, scal);
}

template <typename T>
void launch_dot_rz(Dims d, const double *r, const T *z, double *part, hipStream_t s)
{
    hipLaunchKernelGGL((k_dot_rz<T>), red_grid(d), kBlock, 0, s, d, r, z, part);
}


template <typename T>
int launch_dir_apply(Dims d, Bc bc, const double *bx, const double *by, const double *bz,
                     const double *rho, const T *z, const typename DirT<T>::type *dold,
                     typename DirT<T>::type *dnew, double *q, double *x, const double *sg,
                     const double *scal, int mode, double ih2, double *part, size_t pstride,
                     hipStream_t s)
{
    using D = typename DirT<T>::type;
    // 2 x 2 cells per thread where the grid and the iterate allow pairs
    const bool quad = d.nx % 2 == 0 && d.ny % 2 == 0 && ((uintptr_t)x & 15) == 0;
    const dim3 g = quad ? dim3((d.nx / 2 + BX - 1) / BX, (d.ny / 2 + BY - 1) / BY,
                               (d.nz + RZ - 1) / RZ)
                        : red_grid(d);
    auto go = [&](auto kern) {
        PP_LAUNCH(kern, g, kBlock, 0, s, d, bc, bx, by, bz, rho, z, dold, dnew, q, x, sg,
                  scal, ih2, part, pstride);
    };
    auto by_mode = [&](auto r) {
        constexpr bool RH = decltype(r)::value;
        if (quad) {
            if (mode == DIR_FIRST)
                go(k_dir_apply2<T, D, DIR_FIRST, RH>);
            else if (mode == DIR_HOLD)
                go(k_dir_apply2<T, D, DIR_HOLD, RH>);
            else
                go(k_dir_apply2<T, D, DIR_TWO, RH>);
        } else {
            if (mode == DIR_FIRST)
                go(k_dir_apply<T, D, DIR_FIRST, RH>);
            else if (mode == DIR_HOLD)
                go(k_dir_apply<T, D, DIR_HOLD, RH>);
            else
                go(k_dir_apply<T, D, DIR_TWO, RH>);
        }
    };
    if (rho)
        by_mode(std::true_type{});
    else
        by_mode(std::false_type{});
    return (int)grid_blocks(g);
}

template <typename T>
void launch_pcg_update(Dims d, const double *q, double *r, T *rT, const double *scal, double *part,
                       hipStream_t s)
{
    PP_LAUNCH((k_pcg_update<T>), red_grid(d), kBlock, 0, s, d, q, r, rT, scal, part);
}

template <typename D>
void launch_axpy_dir(size_t n, const D *dv, const D *dv_prev, double *x, const double *scal,
                     hipStream_t s)
{
    const uintptr_t al = (uintptr_t)dv | (uintptr_t)dv_prev | (uintptr_t)x;
    if (n % 4 == 0 && (al & 15) == 0)
        hipLaunchKernelGGL((k_axpy_dir4<D>), flat_grid(n / 4), dim3(256), 0, s, n / 4, dv, dv_prev, x,
                           scal);
    else
        hipLaunchKernelGGL((k_axpy_dir<D>), flat_grid(n), dim3(256), 0, s, n, dv, dv_prev, x, scal);
}
template void launch_axpy_dir<double>(size_t, const double *, const double *, double *,
                                      const double *, hipStream_t);
template void launch_axpy_dir<float>(size_t, const float *, const float *, double *,
                                     const double *, hipStream_t);

void launch_sub_mean(size_t n, double *x, const double *scal, int slot, const unsigned char *act,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_mean, flat_grid(n), dim3(256), 0, s, n, x, scal, slot, act);
}

// explicit instantiations for the three storage types
#define PP_INSTANTIATE(T)                                                                        \
    template void launch_rbgs<T>(Dims, Bc, const T *, const T *, const T *, const T *, T *,     \
                                 const T *, double, double, int, bool, bool, hipStream_t);      \
    template void launch_resid_restrict<T>(Dims, Bc, const T *, const T *, const T *, const T *, \
                                           const T *, const T *, T *, double, hipStream_t);     \
    template void launch_prolong<T>(Dims, Bc, const T *, T *, const unsigned *, hipStream_t);    \
    template int launch_load_coeffs<T>(Dims, Bc, const double *const[3], double *const[3],      \
                                       T *const[3], double *const[3], unsigned *, double *,     \
                                       hipStream_t, T *const[3]);                               \
    template int launch_load_density<T>(Dims, Bc, const double *, double *const[3], T *const[3], \
                                        double *const[3], double *, unsigned *, double *,       \
                                        hipStream_t);                                           \
    template void launch_coarsest<T>(int, const double *, const T *, T *, hipStream_t);         \
    template void launch_tail<T>(int, const Dims *, const double *, const void *const (*)[3],   \
                                 void *const *, void *const *, const void *const *,             \
                                 const unsigned *const *, Bc, int, int, double, const double *, \
                                 int, bool, hipStream_t);                                       \
    template void launch_convert<T>(size_t, const double *, T *, hipStream_t);                  \
    template int launch_convert_scaled<T>(size_t, const double *, double, double, T *, double *, \
                                          int, hipStream_t);                                    \
    template void launch_to_double<T>(size_t, const T *, double *, hipStream_t);                \
    template void launch_residual_T<T>(Dims, Bc, const double *, const double *, const double *, \
                                       const double *, const double *, const double *,          \
                                       const double *, const unsigned char *, T *, double,      \
                                       double *, hipStream_t);                                  \
    template void launch_scale_T<T>(size_t, const double *, T *, const double *, hipStream_t);  \
    template void launch_axpy_T<T>(size_t, const T *, double *, const double *, hipStream_t);   \
    template void launch_dot_rz<T>(Dims, const double *, const T *, double *, hipStream_t);     \
    template int launch_dir_apply<T>(Dims, Bc, const double *, const double *, const double *,  \
                                      const double *, const T *,                                \
                                      const typename DirT<T>::type *,                           \
                                      typename DirT<T>::type *, double *, double *,             \
                                      const double *, const double *, int, double, double *,    \
                                      size_t, hipStream_t);                                     \
    template void launch_pcg_update<T>(Dims, const double *, double *, T *, const double *,     \
                                       double *, hipStream_t);

PP_INSTANTIATE(double)
PP_INSTANTIATE(float)
PP_INSTANTIATE(_Float16)

}  // namespace pp
