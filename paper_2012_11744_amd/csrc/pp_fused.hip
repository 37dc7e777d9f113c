// pp_fused.hip -- the fused red-black Gauss-Seidel sweep (gfx950), the
// dominant kernel of the V-cycle: both colours of one sweep in one pass over
// the level, out of place.
//
// The update is the seven-point Gauss-Seidel step of Sec. 3.7.1 with
// relaxation 1 (the SOR iteration of that section with omega = 1), cells
// coloured red ((i+j+k) even) and black; walls (Sec. 3.8) zero the link
// coefficient of the wall face.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "pp_device.h"
#include "pp_internal.h"

namespace pp {

// ---------------------------------------------------------------------------
// Fused red-black Gauss-Seidel sweep (both colours in one pass, out of place).
//
// A block owns an FTX x FTY tile of an x-y plane and marches along z through a
// chunk of planes [k0, k1).  Each thread owns one x-pair of cells (2p, 2p+1)
// of one row: at every plane exactly one cell of a pair has each colour.  At
// step k a thread updates the first-colour cell of its pair in plane k and
// publishes it in an LDS plane slot; after one barrier the tile threads
// update the second-colour cell of plane k-1 from the slots (in-plane
// neighbours) and from their own registers (the z neighbours, which are the
// first-colour cells of the same pair in planes k-2 and k), and store the
// finished pair of plane k-1.
//
// The threads of a one-pair / one-row ring around the tile, and the planes
// k0-1 and k1, recompute first-colour values that belong to neighbouring
// tiles and chunks from the same inputs, so blocks never read each other's
// output (e_in is read only, e_out written only) and every cell gets the
// update of a red-black sweep.  Every input cell is fetched from memory once
// per sweep apart from the ring.
//
// The step has no data-dependent branches: every thread of the layout
// computes the first-colour cell of its pair, reading in-plane neighbours
// from LDS at a column chosen by the pair's colour parity; ring rows also
// publish the row beyond them (two extra LDS rows), padding columns hold
// zeros, and x-wall faces are zeroed as they are published.  Each plane is
// read through buffer resources: a missing plane has an empty range, and an
// inactive thread or a y-wall face uses an offset past the range, so those
// values arrive as zero from the hardware range check and nothing is masked
// after the load.  The loads of plane k+1+FPD therefore stay in flight across
// FPD steps; the loop is unrolled by the buffer rotation period so no buffer
// with loads in flight is copied.
// ---------------------------------------------------------------------------
constexpr int FTX = 128;                // tile width in cells (64 pairs)
constexpr int FTY = 8;                  // tile height in rows
constexpr int FPX = FTX / 2 + 2;        // pairs per row including the ring pairs
constexpr int FRY = FTY + 2;            // thread rows including the ring rows
constexpr int FTHREADS = (FPX * FRY + 63) / 64 * 64;   // whole waves
constexpr int FLW = FTX + 8;            // LDS row: cells i0-4 .. i0+FTX+3
constexpr int FLR = FTY + 4;            // LDS rows: j0-2 .. j0+FTY+1

// Planes of loads in flight beyond plane k+1, per storage type: two for FP32
// (its loads are small, so it needs more of them in flight); one for FP64,
// whose registers would otherwise spill, and for FP16 (measured best at one).
template <typename T>
struct FusedDepth {
    static constexpr int value = sizeof(T) == 4 ? 2 : 1;
};

// Inputs of one thread's pair at one plane, as loaded (storage precision).
// eo / byo: e_in and beta_y of the row beyond an outermost ring row (zero
// for the other threads, which read no such row).  Values a thread must
// treat as zero (inactive thread, missing plane, wall faces of y and z)
// arrive as zero from the buffer range check.
template <typename T>
struct PairIn {
    using T2 = typename Vec2<T>::type;
    T2 e, r, bx, by, bz, eo, byo;
    T2 sg;                     // diagonal term (general operator only)
};

// Buffer resource over one plane: loads at byte offsets >= `bytes` return
// zero and stores there are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ typename Vec2<T>::type ld_pair(__amdgpu_buffer_rsrc_t rs, unsigned off)
{
    using T2 = typename Vec2<T>::type;
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    else if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    else
        return __builtin_bit_cast(T2, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
}

template <typename T>
__device__ __forceinline__ void st_pair(__amdgpu_buffer_rsrc_t rs, unsigned off,
                                        typename Vec2<T>::type v)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b128(
            __builtin_bit_cast(unsigned __attribute__((ext_vector_type(4))), v), rs, off, 0, 0);
    else if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(unsigned __attribute__((ext_vector_type(2))), v), rs, off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, off, 0, 0);
}

// an offset past every plane (planes of a fused sweep stay below 2^31 bytes)
constexpr unsigned OFF_NONE = 0x80000000u;

__device__ __forceinline__ int slot3(int k) { return ((k % 3) + 3) % 3; }

// The Gauss-Seidel quotient.  FP32 arithmetic (FP32 and FP16 storage) takes
// the hardware reciprocal (within 1 ulp) times the numerator: the smoother
// only has to reduce the error, and its result is a preconditioner that the
// FP64 outer iteration corrects; FP64 keeps the exact quotient.
__device__ __forceinline__ float gs_quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double gs_quot(double a, double b) { return a / b; }

// Block id -> (tile x, tile y, chunk), spreading contiguous ranges of tiles over
// the 8 XCDs: consecutive workgroups are dispatched round-robin to the XCDs,
// so workgroup b is given logical tile (b % 8) * (n / 8) + b / 8, which keeps
// neighbouring tiles (which share halo lines) in one XCD's L2.  The grid is
// (tiles of a plane) x (z chunks); b is the linear workgroup index.
__device__ __forceinline__ void xcd_tile(unsigned tx_tiles, unsigned ty_tiles, int &bxi, int &byi,
                                         int &bzi)
{
    const unsigned nb = gridDim.x * gridDim.y;
    unsigned b = blockIdx.x + gridDim.x * blockIdx.y;
    const unsigned full = nb & ~7u;
    if (b < full)
        b = (b & 7u) * (full >> 3) + (b >> 3);
    bxi = (int)(b % tx_tiles);
    byi = (int)((b / tx_tiles) % ty_tiles);
    bzi = (int)(b / (tx_tiles * ty_tiles));
}

// SIG: the general operator's diagonal term, stored as h^2 sigma, is read
// with the other inputs and added to the diagonal.  In every variant a cell with a
// zero diagonal (no open face, no diagonal term) is excluded and gets 0.
// WHOLE: the march runs whole blocks of its unroll length (see the loop).
// om: the over-relaxation of eq. beta_pressure, e <- (1 - om) e + om e_GS
// (ZERO: the old value is 0).
template <typename T, bool ZERO, bool SIG, bool WHOLE>
__global__ __launch_bounds__(FTHREADS) void k_rbgs_fused(Dims d, Bc bc, const T *__restrict__ bx,
                                                         const T *__restrict__ by,
                                                         const T *__restrict__ bz,
                                                         const T *__restrict__ r,
                                                         const T *__restrict__ ein,
                                                         T *__restrict__ eout,
                                                         const T *__restrict__ sg,
                                                         typename Acc<T>::type h2,
                                                         typename Acc<T>::type om, int c0, int kz,
                                                         unsigned tx_tiles, unsigned ty_tiles)
{
    using C = typename Acc<T>::type;
    using T2 = typename Vec2<T>::type;
    const C om1 = C(1) - om;
    constexpr int FPD = FusedDepth<T>::value;   // planes of loads in flight beyond k+1
    constexpr int FNB = FPD + 3;                // input buffers: k-1, k, k+1 and those in flight
    // LDS: e_in, beta_x and beta_y of planes k and k+1 (two slots) for the
    // in-plane neighbours, and the first-colour values of planes k-2..k
    __shared__ C SE[2][FLR][FLW];
    __shared__ C SX[2][FLR][FLW];
    __shared__ C SY[2][FLR][FLW];
    __shared__ C RED[3][FLR][FLW];
    int bxi, byi, bzi;
    xcd_tile(tx_tiles, ty_tiles, bxi, byi, bzi);
    const int i0 = bxi * FTX, j0 = byi * FTY;
    const int k0 = bzi * kz;
    const int k1 = min(k0 + kz, d.nz);

    const int tid = threadIdx.x;
    const bool in_layout = tid < FPX * FRY;
    // threads past the layout shadow thread 0 (inactive: they publish and
    // store nothing, and their LDS reads stay inside the arrays)
    const int tl = in_layout ? tid : 0;
    const int pl = tl % FPX - 1;      // pair within the tile; -1 and FTX/2 are ring pairs
    const int rl = tl / FPX - 1;      // row within the tile; -1 and FTY are ring rows
    int x = i0 + 2 * pl;
    int j = j0 + rl;
    // the pair / row just past the grid's end is the periodic wrap: ring only
    const bool ringx = pl < 0 || pl >= FTX / 2 || x == d.nx;
    const bool ringy = rl < 0 || rl >= FTY || j == d.ny;
    bool act = in_layout;             // holds a pair of the grid
    if (x < 0) {
        if (bc.x) act = false; else x += d.nx;
    } else if (x >= d.nx) {
        if (bc.x || x > d.nx) act = false; else x = 0;
    }
    if (j < 0) {
        if (bc.y) act = false; else j += d.ny;
    } else if (j >= d.ny) {
        if (bc.y || j > d.ny) act = false; else j = 0;
    }
    if (!act) {
        x = 0;
        j = 0;
    }
    const bool owned = act && !ringx && !ringy;
    const bool dn_row = act && rl < 0;                 // publishes the row below it
    const bool up_row = act && ringy && rl >= 0;       // publishes the row above it
    const int jm = (j == 0) ? d.ny - 1 : j - 1;
    const int jp = (j == d.ny - 1) ? 0 : j + 1;
    const bool wyl = bc.y && j == 0, wyh = bc.y && j == d.ny - 1;
    const bool wxl = bc.x && x == 0;
    const int jo = dn_row ? jm : (up_row ? jp : j);
    const bool zo = up_row ? wyh : wyl;   // the y faces published in row lyo are walls
    const bool beyond = dn_row || up_row;   // only these threads read the row beyond
    // byte offsets of the pair within a plane; OFF_NONE reads zero (and, for
    // the row beyond, spares the other threads a load of their own row)
    const unsigned oc0 = (unsigned)(((size_t)j * d.nx + x) * sizeof(T));
    const unsigned oo0 = (unsigned)(((size_t)jo * d.nx + x) * sizeof(T));
    const unsigned oc = act ? oc0 : OFF_NONE;
    const unsigned oo = (act && beyond) ? oo0 : OFF_NONE;
    const unsigned ocy = (act && !wyl) ? oc0 : OFF_NONE;
    const unsigned ooy = (act && beyond && !zo) ? oo0 : OFF_NONE;
    const unsigned ost = owned ? oc0 : OFF_NONE;
    const unsigned pbytes = (unsigned)((size_t)d.nx * d.ny * sizeof(T));
    const int lx = 2 * pl + 4;        // LDS column of the pair's first cell
    const int ly = rl + 2;            // LDS row of the pair
    const int lyo = dn_row ? ly - 1 : (up_row ? ly + 1 : ly);

    // plane q: its wrapped index, and whether it exists (walls end the grid)
    auto plane = [&](int q, int &qw) -> bool {
        qw = q;
        if (q < 0) {
            if (bc.z) { qw = 0; return false; }
            qw = q + d.nz;
        } else if (q >= d.nz) {
            if (bc.z) { qw = 0; return false; }
            qw = q - d.nz;
        }
        return true;
    };
    auto load_in = [&](int q, PairIn<T> &v) __attribute__((always_inline)) {
        int qw;
        const unsigned nb = plane(q, qw) ? pbytes : 0u;
        const size_t pb = (size_t)qw * pbytes;
        auto rs = [&](const T *base, unsigned n) {
            return plane_rsrc(reinterpret_cast<const char *>(base) + pb, n);
        };
        if (!ZERO) {
            const auto re = rs(ein, nb);
            v.e = ld_pair<T>(re, oc);
            v.eo = ld_pair<T>(re, oo);
        }
        v.r = ld_pair<T>(rs(r, nb), oc);
        v.bx = ld_pair<T>(rs(bx, nb), oc);
        const auto ry = rs(by, nb);
        v.by = ld_pair<T>(ry, ocy);
        v.byo = ld_pair<T>(ry, ooy);
        v.bz = ld_pair<T>(rs(bz, (bc.z && qw == 0) ? 0u : nb), oc);   // the wall below plane 0
        if (SIG)
            v.sg = ld_pair<T>(rs(sg, nb), oc);
    };
    auto pick = [](int o, T2 v) -> C { return C(o ? v.y : v.x); };
    // Only active threads write LDS: the positions of inactive ones (past a
    // wall, past a ragged grid end) keep the zeros of the initial fill, and
    // the row a wrapping ring row publishes beyond itself may be the own row
    // of an inactive thread.
    auto publish = [&](int slot, const PairIn<T> &v) __attribute__((always_inline)) {
        if (!act)
            return;
        if (!ZERO) {
            SE[slot][ly][lx] = C(v.e.x);
            SE[slot][ly][lx + 1] = C(v.e.y);
        }
        SX[slot][ly][lx] = wxl ? C(0) : C(v.bx.x);
        SX[slot][ly][lx + 1] = C(v.bx.y);
        SY[slot][ly][lx] = C(v.by.x);
        SY[slot][ly][lx + 1] = C(v.by.y);
        if (beyond) {
            if (!ZERO) {
                SE[slot][lyo][lx] = C(v.eo.x);
                SE[slot][lyo][lx + 1] = C(v.eo.y);
            }
            SY[slot][lyo][lx] = C(v.byo.x);
            SY[slot][lyo][lx + 1] = C(v.byo.y);
        }
    };

    // padding columns and rows read as zero
    for (int i = tid; i < 2 * FLR * FLW; i += FTHREADS) {
        (&SE[0][0][0])[i] = C(0);
        (&SX[0][0][0])[i] = C(0);
        (&SY[0][0][0])[i] = C(0);
    }
    for (int i = tid; i < 3 * FLR * FLW; i += FTHREADS)
        (&RED[0][0][0])[i] = C(0);

    C red_km2 = C(0), red_km1 = C(0);
    // in-plane faces of the second-colour cell of plane k-1 (read at step k-1)
    C sxl = C(0), sxh = C(0), syl = C(0), syh = C(0);

    // One plane step: inputs of planes k-1 (pm), k (pc), k+1 (pn) resident,
    // plane k+1+FPD (pf) loaded here and left in flight for FPD steps.
    auto step = [&](int k, PairIn<T> &pm, PairIn<T> &pc, PairIn<T> &pn, PairIn<T> &pf)
                    __attribute__((always_inline)) {
        load_in(k + 1 + FPD, pf);
        const int si = k & 1;
        int kw;
        const bool kin = act && plane(k, kw);
        const int o = (c0 + j + k) & 1;   // first-colour cell of the pair in plane k
        // phase A: first colour of plane k
        const int ca = lx + o;
        const C xl = SX[si][ly][ca], xh = SX[si][ly][ca + 1];
        const C yl = SY[si][ly][ca], yh = SY[si][ly + 1][ca];
        const C zl = pick(o, pc.bz), zh = pick(o, pn.bz);
        C diag = (xl + xh) + (yl + yh) + (zl + zh);
        if (SIG)
            diag += pick(o, pc.sg);          // h^2 sigma
        C s = C(0);
        if (!ZERO)
            s = xl * SE[si][ly][ca - 1] + xh * SE[si][ly][ca + 1] + yl * SE[si][ly - 1][ca] +
                yh * SE[si][ly + 1][ca] + zl * pick(o, pm.e) + zh * pick(o, pn.e);
        const C val = gs_quot(s - h2 * pick(o, pc.r), diag);
        // a missing plane (0/0) and an excluded cell (zero diagonal) get 0
        const C rel = ZERO ? om * val : om1 * pick(o, pc.e) + om * val;
        const C red = (kin && diag > C(0)) ? rel : C(0);
        // in-plane faces of this plane's second-colour cell, for phase B at
        // the next step (the slot is overwritten before then)
        const int cb = lx + 1 - o;
        const C nxl = SX[si][ly][cb], nxh = SX[si][ly][cb + 1];
        const C nyl = SY[si][ly][cb], nyh = SY[si][ly + 1][cb];
        if (act)
            RED[slot3(k)][ly][ca] = red;
        publish(si ^ 1, pn);          // plane k+1 for the next step's phase A
        __syncthreads();
        // phase B: second colour of plane k-1 (at the column of this plane's
        // first colour); the store of a thread outside the tile is dropped
        const int kb = k - 1;
        if (kb >= k0 && kb < k1) {
            const int sb = slot3(kb);
            const C bzl = pick(o, pm.bz), bzh = pick(o, pc.bz);
            const C sbv = sxl * RED[sb][ly][ca - 1] + sxh * RED[sb][ly][ca + 1] +
                          syl * RED[sb][ly - 1][ca] + syh * RED[sb][ly + 1][ca] + bzl * red_km2 +
                          bzh * red;
            C dg = (sxl + sxh) + (syl + syh) + (bzl + bzh);
            if (SIG)
                dg += pick(o, pm.sg);
            const C q = gs_quot(sbv - h2 * pick(o, pm.r), dg);
            const C blk = dg > C(0) ? (ZERO ? om * q : om1 * pick(o, pm.e) + om * q) : C(0);
            T2 outv;
            outv.x = static_cast<T>(o ? red_km1 : blk);
            outv.y = static_cast<T>(o ? blk : red_km1);
            st_pair<T>(plane_rsrc(reinterpret_cast<const char *>(eout) + (size_t)kb * pbytes, pbytes),
                       ost, outv);
        }
        red_km2 = red_km1;
        red_km1 = red;
        sxl = nxl;
        sxh = nxh;
        syl = nyl;
        syh = nyh;
    };

    // FNB input buffers rotate through the roles (k-1, k, k+1, and the planes
    // in flight); the loop is unrolled by FNB so no buffer with loads in
    // flight is ever copied.  WHOLE: it runs whole blocks of FNB steps, the
    // last up to FNB - 1 steps past k1 (they store nothing), with one exit
    // test per block, which keeps the loop-carried registers in place across
    // the back edge; an exit after every step makes the compiler copy
    // registers with loads in flight there (waiting for them), which costs
    // less than the extra steps only on short chunks.
    PairIn<T> buf[FNB];
#pragma unroll
    for (int u = 0; u < FNB - 1; ++u)
        load_in(k0 - 2 + u, buf[u]);
    __syncthreads();                  // the zero fill is complete
    publish((k0 - 1) & 1, buf[1]);
    __syncthreads();
    if constexpr (WHOLE) {
        for (int k = k0 - 1; k <= k1; k += FNB) {
#pragma unroll
            for (int u = 0; u < FNB; ++u)
                step(k + u, buf[u % FNB], buf[(u + 1) % FNB], buf[(u + 2) % FNB],
                     buf[(u + FNB - 1) % FNB]);
        }
    } else {
        for (int k = k0 - 1;;) {
#pragma unroll
            for (int u = 0; u < FNB; ++u) {
                step(k, buf[u % FNB], buf[(u + 1) % FNB], buf[(u + 2) % FNB],
                     buf[(u + FNB - 1) % FNB]);
                if (++k > k1)
                    return;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------

// Workgroups of a fused-sweep kernel that the whole GPU holds at once
// (occupancy x CUs), queried once per kernel instantiation and device.  The
// cache lives in the (T, ZERO) instantiation: the two variants of one storage
// type have the same function type but different register counts.
template <typename T, bool ZERO, bool SIG>
static long long fused_slots()
{
    static long long cached[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64)
        dev = 0;
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rbgs_fused<T, ZERO, SIG, false>,
                                                         FTHREADS, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            cus = 256;
        cached[dev] = (long long)per_cu * cus;
    }
    return cached[dev];
}

// Marches of at least this many plane steps run whole blocks of the unroll
// length (the WHOLE variants): the few steps a block runs past the chunk cost
// less there than the register copies at the back edge of the other form.
constexpr int WHOLE_MIN_STEPS = 48;

// Chunk length along z: the smallest chunk (fewest redundant halo planes)
// whose workgroups all fit on the GPU at once, so a sweep runs as a single
// round of resident workgroups with no tail.
static int fused_kz(Dims d, unsigned tiles, long long slots)
{
    long long kz = ((long long)d.nz * tiles + slots - 1) / slots;
    if (kz < 4)
        kz = 4;
    if (kz > d.nz)
        kz = d.nz;
    return (int)kz;
}

template <typename T>
void prepare_fused()
{
    (void)fused_slots<T, true, false>();
    (void)fused_slots<T, false, false>();
    (void)fused_slots<T, true, true>();
    (void)fused_slots<T, false, true>();
}

template <typename T>
void launch_rbgs_fused(Dims d, Bc bc, const T *bx, const T *by, const T *bz, const T *r,
                       const T *ein, T *eout, const T *sg, double h2, double omega,
                       int first_colour, bool zero, hipStream_t s)
{
    using C = typename Acc<T>::type;
    const unsigned tx = (d.nx + FTX - 1) / FTX, ty = (d.ny + FTY - 1) / FTY;
    const long long slots = sg ? (zero ? fused_slots<T, true, true>() : fused_slots<T, false, true>())
                               : (zero ? fused_slots<T, true, false>() : fused_slots<T, false, false>());
    const int kz = fused_kz(d, tx * ty, slots);
    const unsigned tz = (d.nz + kz - 1) / kz;
    const dim3 grid(tx * ty, tz);   // distinct shapes per level in profiles
    const bool whole = kz + 2 >= WHOLE_MIN_STEPS;   // a chunk marches kz + 2 steps
#define PP_FUSED_LAUNCH(Z, S)                                                                  \
    do {                                                                                       \
        if (whole)                                                                             \
            PP_LAUNCH((k_rbgs_fused<T, Z, S, true>), grid, dim3(FTHREADS), 0, s, d, bc, bx,    \
                      by, bz, r, ein, eout, sg, (C)h2, (C)omega, first_colour, kz, tx, ty);    \
        else                                                                                   \
            PP_LAUNCH((k_rbgs_fused<T, Z, S, false>), grid, dim3(FTHREADS), 0, s, d, bc, bx,   \
                      by, bz, r, ein, eout, sg, (C)h2, (C)omega, first_colour, kz, tx, ty);    \
    } while (0)
    if (sg) {
        if (zero)
            PP_FUSED_LAUNCH(true, true);
        else
            PP_FUSED_LAUNCH(false, true);
    } else {
        if (zero)
            PP_FUSED_LAUNCH(true, false);
        else
            PP_FUSED_LAUNCH(false, false);
    }
#undef PP_FUSED_LAUNCH
}

// ---------------------------------------------------------------------------
// Two sweeps in one pass (FP32 arithmetic: FP32 and FP16 storage).
//
// The plane step above, extended by two phases that lag behind it.  At step k
//   A: first colour of plane k, sweep 1 (from e_in, as above);
//   B: second colour of plane k-1, sweep 1;
//   C: first colour of plane k-2, sweep 2, from the finished sweep-1 values;
//   D: second colour of plane k-3, sweep 2, which completes that plane.
// Every phase reads its in-plane neighbours from an LDS plane written one
// step earlier (A from the published inputs, B from A's values, C from B's,
// D from C's) and its z neighbours, the same pair's cells in the planes above
// and below, from registers.  C and D update the same cells as A and B two
// steps before, so they reuse the coefficients, reciprocal diagonal and h^2 r
// that A and B computed, carried in registers.  One barrier per step
// separates A (and the publication of the next plane's inputs) from B, C and
// D.  Each phase consumes one ring cell, so the ring around the tile is two
// pairs wide and three rows deep, and a chunk of output planes [k0, k1) is
// marched from k0-3 to k1+2.  Per cell the pass moves the bytes of one sweep.
// ---------------------------------------------------------------------------
constexpr int GTX = 64;                   // tile width in cells (32 pairs)
constexpr int GTY = 8;                    // tile height in rows
constexpr int GPX = GTX / 2 + 4;          // pairs per row: two ring pairs on each side
constexpr int GRY = GTY + 6;              // rows: three ring rows on each side
constexpr int GTHREADS = (GPX * GRY + 63) / 64 * 64;
constexpr int GLW = GTX + 12;             // LDS row: cells i0-6 .. i0+GTX+5
constexpr int GLR = GTY + 8;              // LDS rows: j0-4 .. j0+GTY+3

// what phase A (B) computed for a cell, for phase C (D) two steps later
struct GsLag {
    float xl, xh, yl, yh, zl, zh;   // link coefficients
    float inv;                      // om / diagonal, or 0 for an excluded cell or missing plane
    float hr;                       // h^2 r
};

// om: the over-relaxation of eq. beta_pressure, folded into the reciprocal
// diagonal that the lag registers carry (inv = om / diag), so every phase
// forms e <- (1 - om) e + inv (sum - h^2 r); the old value of phases A and B
// is e_in (0 in the ZERO pass), that of C and D the sweep-1 value.
// DOT (FP32, regular pass): also the partial sums of r . e_out over each
// workgroup's output cells, r the pass's own right-hand side, products summed
// in FP64 (the outer iteration's residual against the preconditioned one,
// both in units of the V-cycle's scale); part[workgroup].  The h^2 r values
// that phases C and D already carry supply r, so nothing more is loaded.
template <typename T, bool ZERO, bool SIG, bool DOT, bool WHOLE>
__global__ __launch_bounds__(GTHREADS) void k_rbgs_fused2(Dims d, Bc bc, const T *__restrict__ bx,
                                                          const T *__restrict__ by,
                                                          const T *__restrict__ bz,
                                                          const T *__restrict__ r,
                                                          const T *__restrict__ ein,
                                                          T *__restrict__ eout,
                                                          const T *__restrict__ sg, float h2,
                                                          float om, int c0, int kz, unsigned tx_tiles,
                                                          unsigned ty_tiles,
                                                          double *__restrict__ part)
{
    using C = float;
    using T2 = typename Vec2<T>::type;
    // Planes of loads in flight beyond k+1: three for FP32, one for FP16
    // (whose registers then allow two workgroups per CU).  The loop is
    // unrolled by the buffer count FNB; with FP32's six buffers, a multiple
    // of both slot periods (2 and 3), every LDS slot index is a compile-time
    // constant.
    constexpr int FPD = sizeof(T) == 4 ? 3 : 1;
    constexpr int FNB = FPD + 3;
    constexpr bool CT_SLOTS = FNB % 6 == 0;
    static_assert(!DOT || (!ZERO && !SIG), "the dot product rides on regular passes");
    const C om1 = C(1) - om;
    __shared__ C SE[2][GLR][GLW];     // e_in of planes k, k+1
    __shared__ C SX[2][GLR][GLW];     // beta_x of planes k, k+1
    __shared__ C SY[2][GLR][GLW];     // beta_y of planes k, k+1
    __shared__ C RED1[3][GLR][GLW];   // phase A values (sweep 1, first colour)
    __shared__ C BLK1[2][GLR][GLW];   // phase B values (sweep 1, second colour)
    __shared__ C RED2[2][GLR][GLW];   // phase C values (sweep 2, first colour)
    int bxi, byi, bzi;
    xcd_tile(tx_tiles, ty_tiles, bxi, byi, bzi);
    const int i0 = bxi * GTX, j0 = byi * GTY;
    const int k0 = bzi * kz;
    const int k1 = min(k0 + kz, d.nz);
    const int xend = min(i0 + GTX, d.nx), yend = min(j0 + GTY, d.ny);

    const int tid = threadIdx.x;
    const bool in_layout = tid < GPX * GRY;
    const int tl = in_layout ? tid : 0;
    const int pl = tl % GPX - 2;      // pair within the tile; -2, -1 and those past xend are ring
    const int rl = tl / GPX - 3;      // row within the tile; -3..-1 and those past yend are ring
    const int xu = i0 + 2 * pl, ju = j0 + rl;
    int x = xu, j = ju;
    // ring pairs / rows past the grid's end wrap when periodic (at most two
    // pairs, three rows); with walls they hold no cell
    bool act = in_layout;
    if (xu < 0) {
        if (bc.x) act = false; else x = xu + d.nx;
    } else if (xu >= d.nx) {
        if (bc.x || xu >= d.nx + 4) act = false; else x = xu - d.nx;
    }
    if (ju < 0) {
        if (bc.y) act = false; else j = ju + d.ny;
    } else if (ju >= d.ny) {
        if (bc.y || ju >= d.ny + 3) act = false; else j = ju - d.ny;
    }
    if (!act) {
        x = 0;
        j = 0;
    }
    const bool owned = act && pl >= 0 && xu < xend && rl >= 0 && ju < yend;
    const bool dn_row = act && rl == -3;              // publishes the row below it
    const bool up_row = act && ju == yend + 2;        // publishes the row above it
    const int jm = (j == 0) ? d.ny - 1 : j - 1;
    const int jp = (j == d.ny - 1) ? 0 : j + 1;
    const bool wyl = bc.y && j == 0, wyh = bc.y && j == d.ny - 1;
    const bool wxl = bc.x && x == 0;
    const int jo = dn_row ? jm : (up_row ? jp : j);
    const bool zo = up_row ? wyh : wyl;
    const bool beyond = dn_row || up_row;   // only these threads read the row beyond
    const unsigned oc0 = (unsigned)(((size_t)j * d.nx + x) * sizeof(T));
    const unsigned oo0 = (unsigned)(((size_t)jo * d.nx + x) * sizeof(T));
    const unsigned oc = act ? oc0 : OFF_NONE;
    const unsigned oo = (act && beyond) ? oo0 : OFF_NONE;
    const unsigned ocy = (act && !wyl) ? oc0 : OFF_NONE;
    const unsigned ooy = (act && beyond && !zo) ? oo0 : OFF_NONE;
    const unsigned ost = owned ? oc0 : OFF_NONE;
    const unsigned pbytes = (unsigned)((size_t)d.nx * d.ny * sizeof(T));
    const int lx = 2 * pl + 6;        // LDS column of the pair's first cell
    const int ly = rl + 4;            // LDS row of the pair
    const int lyo = dn_row ? ly - 1 : (up_row ? ly + 1 : ly);

    // plane q: its wrapped index, and whether it exists (walls end the grid);
    // selects rather than branches (q is within four planes of the grid)
    auto plane = [&](int q, int &qw) -> bool {
        const bool lo = q < 0, hi = q >= d.nz;
        qw = lo ? q + d.nz : (hi ? q - d.nz : q);
        const bool ok = !(bc.z && (lo || hi));
        qw = ok ? qw : 0;
        return ok;
    };
    auto load_in = [&](int q, PairIn<T> &v) __attribute__((always_inline)) {
        int qw;
        const unsigned nb = plane(q, qw) ? pbytes : 0u;
        const size_t pb = (size_t)qw * pbytes;
        auto rs = [&](const T *base, unsigned n) {
            return plane_rsrc(reinterpret_cast<const char *>(base) + pb, n);
        };
        if (!ZERO) {
            const auto re = rs(ein, nb);
            v.e = ld_pair<T>(re, oc);
            v.eo = ld_pair<T>(re, oo);
        }
        v.r = ld_pair<T>(rs(r, nb), oc);
        v.bx = ld_pair<T>(rs(bx, nb), oc);
        const auto ry = rs(by, nb);
        v.by = ld_pair<T>(ry, ocy);
        v.byo = ld_pair<T>(ry, ooy);
        v.bz = ld_pair<T>(rs(bz, (bc.z && qw == 0) ? 0u : nb), oc);
        if (SIG)
            v.sg = ld_pair<T>(rs(sg, nb), oc);
    };
    auto pick = [](int o, T2 v) -> C { return C(o ? v.y : v.x); };
    auto publish = [&](int slot, const PairIn<T> &v) __attribute__((always_inline)) {
        if (!act)
            return;
        if (!ZERO) {
            SE[slot][ly][lx] = C(v.e.x);
            SE[slot][ly][lx + 1] = C(v.e.y);
        }
        SX[slot][ly][lx] = wxl ? C(0) : C(v.bx.x);
        SX[slot][ly][lx + 1] = C(v.bx.y);
        SY[slot][ly][lx] = C(v.by.x);
        SY[slot][ly][lx + 1] = C(v.by.y);
        if (beyond) {
            if (!ZERO) {
                SE[slot][lyo][lx] = C(v.eo.x);
                SE[slot][lyo][lx + 1] = C(v.eo.y);
            }
            SY[slot][lyo][lx] = C(v.byo.x);
            SY[slot][lyo][lx + 1] = C(v.byo.y);
        }
    };

    for (int i = tid; i < 2 * GLR * GLW; i += GTHREADS) {
        (&SE[0][0][0])[i] = C(0);
        (&SX[0][0][0])[i] = C(0);
        (&SY[0][0][0])[i] = C(0);
        (&BLK1[0][0][0])[i] = C(0);
        (&RED2[0][0][0])[i] = C(0);
    }
    for (int i = tid; i < 3 * GLR * GLW; i += GTHREADS)
        (&RED1[0][0][0])[i] = C(0);

    // own-pair values of earlier planes: A's of k-1, k-2; B's of k-2, k-3;
    // C's of k-3, k-4
    C red_km1 = C(0), red_km2 = C(0);
    C blk_km1 = C(0), blk_km2 = C(0);
    C r2_km1 = C(0), r2_km2 = C(0);
    C sxl = C(0), sxh = C(0), syl = C(0), syh = C(0);
    GsLag a1{}, a2{}, b1{}, b2{};
    // DOT: h^2 r of C's cell of the previous step (the first-colour cell of
    // the plane phase D completes), and the sum of h^2 r e_out
    C hrc = C(0);
    double dacc = 0.0;

    // LDS slots are counted from the first plane of the march, kb = k0 - 3:
    // plane k's inputs sit in slot (k - kb) mod 2, its phase-A values in slot
    // (k - kb) mod 3; u is the unrolled step index, (k - kb) mod FNB
    const int kb = k0 - 3;
    const int p0 = (c0 + j + kb) & 1;
    // waves that hold only outer ring rows, whose phase C and D values no
    // thread reads, skip those phases
    const bool cdw = __any(in_layout && rl >= -1 && rl <= GTY);
    auto step = [&](int k, int u, PairIn<T> &pm, PairIn<T> &pc, PairIn<T> &pn, PairIn<T> &pf)
                    __attribute__((always_inline)) {
        load_in(k + 1 + FPD, pf);
        const int st = CT_SLOTS ? u : k - kb;
        const int si = st & 1;
        const int s3 = CT_SLOTS ? u % 3 : slot3(st);
        int kw;
        const bool kin = act && plane(k, kw);
        const int o = p0 ^ (st & 1);      // first-colour cell of the pair in plane k
        const int ca = lx + o;            // the cell every phase of this step updates
        // phase A: first colour of plane k, sweep 1
        const C xl = SX[si][ly][ca], xh = SX[si][ly][ca + 1];
        const C yl = SY[si][ly][ca], yh = SY[si][ly + 1][ca];
        const C zl = pick(o, pc.bz), zh = pick(o, pn.bz);
        C diag = (xl + xh) + (yl + yh) + (zl + zh);
        if (SIG)
            diag += pick(o, pc.sg);
        C s = C(0);
        if (!ZERO)
            s = xl * SE[si][ly][ca - 1] + xh * SE[si][ly][ca + 1] + yl * SE[si][ly - 1][ca] +
                yh * SE[si][ly + 1][ca] + zl * pick(o, pm.e) + zh * pick(o, pn.e);
        const C inva = (kin && diag > C(0)) ? om * __builtin_amdgcn_rcpf(diag) : C(0);
        const C hra = h2 * pick(o, pc.r);
        C red = (s - hra) * inva;
        if (!ZERO) {
            red = om1 * pick(o, pc.e) + red;
            if (SIG)
                red = inva == C(0) ? C(0) : red;   // an excluded cell stays 0
        }
        const int cb = lx + 1 - o;
        const C nxl = SX[si][ly][cb], nxh = SX[si][ly][cb + 1];
        const C nyl = SY[si][ly][cb], nyh = SY[si][ly + 1][cb];
        if (act)
            RED1[s3][ly][ca] = red;
        publish(si ^ 1, pn);
        __syncthreads();
        // The in-plane neighbours of phases B, C and D were all written before
        // this barrier (A's of plane k-1 in this step, B's of plane k-2 and C's
        // of plane k-3 in the previous one), and none is overwritten below, so
        // all twelve LDS reads are issued at once.
        const int sb = s3 == 0 ? 2 : s3 - 1;
        const C bw = RED1[sb][ly][ca - 1], be = RED1[sb][ly][ca + 1];
        const C bs = RED1[sb][ly - 1][ca], bn = RED1[sb][ly + 1][ca];
        C cw = C(0), ce = C(0), cs = C(0), cn = C(0), dw = C(0), de = C(0), ds = C(0), dn = C(0);
        if (cdw) {
            cw = BLK1[si][ly][ca - 1];
            ce = BLK1[si][ly][ca + 1];
            cs = BLK1[si][ly - 1][ca];
            cn = BLK1[si][ly + 1][ca];
            dw = RED2[si ^ 1][ly][ca - 1];
            de = RED2[si ^ 1][ly][ca + 1];
            ds = RED2[si ^ 1][ly - 1][ca];
            dn = RED2[si ^ 1][ly + 1][ca];
        }
        // phase B: second colour of plane k-1, sweep 1
        const C bzl = pick(o, pm.bz), bzh = pick(o, pc.bz);
        C dg = (sxl + sxh) + (syl + syh) + (bzl + bzh);
        if (SIG)
            dg += pick(o, pm.sg);
        const C invb = dg > C(0) ? om * __builtin_amdgcn_rcpf(dg) : C(0);
        const C hrb = h2 * pick(o, pm.r);
        C blk = (sxl * bw + sxh * be + syl * bs + syh * bn + bzl * red_km2 + bzh * red - hrb) * invb;
        if (!ZERO) {
            blk = om1 * pick(o, pm.e) + blk;
            if (SIG)
                blk = invb == C(0) ? C(0) : blk;
        }
        if (act)
            BLK1[si ^ 1][ly][ca] = blk;
        C red2 = C(0);
        if (cdw) {
            // phase C: first colour of plane k-2, sweep 2 (A's cell of step k-2)
            red2 = om1 * red_km2 + (a2.xl * cw + a2.xh * ce + a2.yl * cs + a2.yh * cn +
                                    a2.zl * blk_km2 + a2.zh * blk - a2.hr) *
                                       a2.inv;
            if (act)
                RED2[si][ly][ca] = red2;
            // phase D: second colour of plane k-3, sweep 2 (B's cell of step k-2)
            const C blk2 = om1 * blk_km2 + (b2.xl * dw + b2.xh * de + b2.yl * ds + b2.yh * dn +
                                            b2.zl * r2_km2 + b2.zh * red2 - b2.hr) *
                                               b2.inv;
            const int kd = k - 3;
            if (kd >= k0 && kd < k1) {
                T2 outv;
                outv.x = static_cast<T>(o ? r2_km1 : blk2);
                outv.y = static_cast<T>(o ? blk2 : r2_km1);
                st_pair<T>(
                    plane_rsrc(reinterpret_cast<const char *>(eout) + (size_t)kd * pbytes, pbytes),
                    ost, outv);
                if (DOT && owned)
                    dacc += static_cast<double>(hrc) * static_cast<double>(r2_km1) +
                            static_cast<double>(b2.hr) * static_cast<double>(blk2);
            }
        }
        red_km2 = red_km1;
        red_km1 = red;
        blk_km2 = blk_km1;
        blk_km1 = blk;
        r2_km2 = r2_km1;
        r2_km1 = red2;
        if (DOT)
            hrc = a2.hr;
        a2 = a1;
        a1 = GsLag{xl, xh, yl, yh, zl, zh, inva, hra};
        b2 = b1;
        b1 = GsLag{sxl, sxh, syl, syh, bzl, bzh, invb, hrb};
        sxl = nxl;
        sxh = nxh;
        syl = nyl;
        syh = nyh;
    };

    PairIn<T> buf[FNB];
#pragma unroll
    for (int u = 0; u < FNB - 1; ++u)
        load_in(k0 - 4 + u, buf[u]);
    __syncthreads();                  // the zero fill is complete
    publish(0, buf[1]);
    __syncthreads();
    if constexpr (WHOLE) {
        // whole blocks of FNB steps, the last up to FNB - 1 steps past k1 + 2
        // (they store nothing), as in the single sweep.  FP16 does not take
        // this form: its registers would then allow one workgroup per CU
        // instead of two.
        for (int k = kb; k <= k1 + 2; k += FNB) {
#pragma unroll
            for (int u = 0; u < FNB; ++u)
                step(k + u, u, buf[u % FNB], buf[(u + 1) % FNB], buf[(u + 2) % FNB],
                     buf[(u + FNB - 1) % FNB]);
        }
    } else {
        for (int k = kb, more = 1; more;) {
#pragma unroll
            for (int u = 0; u < FNB; ++u) {
                step(k, u, buf[u % FNB], buf[(u + 1) % FNB], buf[(u + 2) % FNB],
                     buf[(u + FNB - 1) % FNB]);
                if (++k > k1 + 2) {
                    more = 0;
                    break;
                }
            }
        }
    }
    if (DOT) {
        __shared__ double wsum[GTHREADS / 64];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            dacc += __shfl_xor(dacc, o, 64);
        if ((tid & 63) == 0)
            wsum[tid >> 6] = dacc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < GTHREADS / 64; ++w)
                t += wsum[w];
            part[blockIdx.x + gridDim.x * blockIdx.y] = t / static_cast<double>(h2);
        }
    }
}

template <typename T, bool ZERO, bool SIG, bool DOT>
static long long fused2_slots()
{
    static long long cached[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64)
        dev = 0;
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                         k_rbgs_fused2<T, ZERO, SIG, DOT, false>,
                                                         GTHREADS, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            cus = 256;
        cached[dev] = (long long)per_cu * cus;
    }
    return cached[dev];
}

template <typename T>
void prepare_fused2()
{
    (void)fused2_slots<T, true, false, false>();
    (void)fused2_slots<T, false, false, false>();
    (void)fused2_slots<T, true, true, false>();
    (void)fused2_slots<T, false, true, false>();
    if constexpr (std::is_same<T, float>::value)
        (void)fused2_slots<T, false, false, true>();
}

template <typename T>
int launch_rbgs_fused2(Dims d, Bc bc, const T *bx, const T *by, const T *bz, const T *r,
                       const T *ein, T *eout, const T *sg, double h2, double omega,
                       int first_colour, bool zero, hipStream_t s, double *part)
{
    const unsigned tx = (d.nx + GTX - 1) / GTX, ty = (d.ny + GTY - 1) / GTY;
    // the fused dot product: FP32 regular passes without a diagonal term
    const bool dot = part && std::is_same<T, float>::value && !zero && !sg;
    long long slots;
    if (dot)
        slots = fused2_slots<T, false, false, std::is_same<T, float>::value>();
    else
        slots = sg ? (zero ? fused2_slots<T, true, true, false>()
                           : fused2_slots<T, false, true, false>())
                   : (zero ? fused2_slots<T, true, false, false>()
                           : fused2_slots<T, false, false, false>());
    // Chunk length: the shortest that keeps every workgroup resident at once
    // (a single round), but at least two planes.  A chunk marches six planes
    // beyond its own, recomputed; on small levels, whose workgroups leave most
    // CUs idle, short chunks cost no time and shorten the march, which sets
    // the pass's duration there.  The pass that forms the dot product keeps
    // chunks of at least 8 planes, so that its workgroup partials stay within
    // the reduction buffer (sized for the grid of the reduction kernels).
    long long kzl = ((long long)d.nz * tx * ty + slots - 1) / slots;
    const int kmin = dot ? 8 : 2;
    if (kzl < kmin)
        kzl = kmin;
    if (kzl > d.nz)
        kzl = d.nz;
    const int kz = (int)kzl;
    const unsigned tz = (d.nz + kz - 1) / kz;
    const dim3 grid(tx * ty, tz);
    // a chunk marches kz + 6 steps; FP16 keeps the exit after every step
    const bool whole = std::is_same<T, float>::value && kz + 6 >= WHOLE_MIN_STEPS;
#define PP_FUSED2_LAUNCH(Z, S, D)                                                              \
    do {                                                                                       \
        if (whole)                                                                             \
            PP_LAUNCH((k_rbgs_fused2<T, Z, S, D, std::is_same<T, float>::value>), grid,        \
                      dim3(GTHREADS), 0, s, d, bc, bx, by, bz, r, ein, eout, sg, (float)h2,    \
                      (float)omega, first_colour, kz, tx, ty, part);                           \
        else                                                                                   \
            PP_LAUNCH((k_rbgs_fused2<T, Z, S, D, false>), grid, dim3(GTHREADS), 0, s, d, bc,   \
                      bx, by, bz, r, ein, eout, sg, (float)h2, (float)omega, first_colour, kz, \
                      tx, ty, part);                                                           \
    } while (0)
    if (dot) {
        if constexpr (std::is_same<T, float>::value)
            PP_FUSED2_LAUNCH(false, false, true);
        return (int)(grid.x * grid.y);
    }
    if (sg) {
        if (zero)
            PP_FUSED2_LAUNCH(true, true, false);
        else
            PP_FUSED2_LAUNCH(false, true, false);
    } else {
        if (zero)
            PP_FUSED2_LAUNCH(true, false, false);
        else
            PP_FUSED2_LAUNCH(false, false, false);
    }
#undef PP_FUSED2_LAUNCH
    return 0;
}

template void prepare_fused2<float>();
template void prepare_fused2<_Float16>();
template int launch_rbgs_fused2<float>(Dims, Bc, const float *, const float *, const float *,
                                       const float *, const float *, float *, const float *, double,
                                       double, int, bool, hipStream_t, double *);
template int launch_rbgs_fused2<_Float16>(Dims, Bc, const _Float16 *, const _Float16 *,
                                          const _Float16 *, const _Float16 *, const _Float16 *,
                                          _Float16 *, const _Float16 *, double, double, int, bool,
                                          hipStream_t, double *);

#define PP_INSTANTIATE_FUSED(T)                                                                  \
    template void prepare_fused<T>();                                                           \
    template void launch_rbgs_fused<T>(Dims, Bc, const T *, const T *, const T *, const T *,    \
                                       const T *, T *, const T *, double, double, int, bool,     \
                                       hipStream_t);

PP_INSTANTIATE_FUSED(double)
PP_INSTANTIATE_FUSED(float)
PP_INSTANTIATE_FUSED(_Float16)

}  // namespace pp
