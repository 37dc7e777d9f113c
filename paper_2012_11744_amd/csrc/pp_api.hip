// pp_api.hip -- host driver and C ABI of the pressure-projection library.
//
// pp_solve runs an FP64 outer iteration (flexible preconditioned conjugate
// gradients by default, or defect correction) around one geometric-multigrid
// V-cycle per iteration (the paper's in-code multigrid, Sec. 3.7.3; red-black
// Gauss-Seidel smoothing, Sec. 3.7.1).  The V-cycle runs in FP64, or in FP32
// (FP16 storage as a variant) on a right-hand side normalised by the RMS of
// the current residual; the outer residual, the coarsest-grid solve and the
// projection stay FP64.  Convergence is checked on the relative L2 norm of
// the residual (the paper lets the user pick L1, L2 or Linf, Sec. 3.7.2),
// read back once per outer iteration.
#include <hip/hip_runtime.h>

#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "pp.h"
#include "pp_internal.h"
#include "pp_kernels.h"

using namespace pp;

namespace {

constexpr int MAXLEV = 24;
constexpr int COARSEST_MAX = 1024;
constexpr int STAGNATED = 1;   // internal code: outer loop stopped improving
constexpr int CONVERGED = 2;   // internal code: the residual reached the tolerance

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define PP_HIP(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(PP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));            \
    } while (0)

#define PP_TRY(call)                                                                            \
    do {                                                                                        \
        int rc_ = (call);                                                                       \
        if (rc_ != PP_OK)                                                                       \
            return rc_;                                                                         \
    } while (0)

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(PP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return PP_OK;
}

enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2 };

size_t storage_bytes(int st) { return st == ST_F64 ? 8 : (st == ST_F32 ? 4 : 2); }

struct LevelBuf {
    Dims d;
    double h;
    void *b[3];
    void *e;      // correction, ping-pong pair with e2 (sweeps are out of place)
    void *e2;
    void *r;
    void *s;      // diagonal term of the general operator (storage type), or null
    void *cur;    // whichever of e / e2 holds the current correction
};

struct Hier {
    int st = ST_F64;
    int nlev = 0;
    bool present = false;
    LevelBuf lev[MAXLEV];
    int tail = 0;                            // first level of the single-workgroup tail
    hipGraphExec_t coarse_exec = nullptr;   // levels 1 .. L-1 of the cycle
};

struct EventPair {
    hipEvent_t a, b;
    int kind;
};

}  // namespace

// host copies of the scalar array: the S_NSLOTS values, then the ticket the
// publishing kernel writes after them
constexpr int HSLOT = S_NSLOTS + 1;

struct pp_ctx {
    pp_grid grid;
    pp_opts opts;
    hipStream_t stream;
    Dims d;
    Bc bc;
    size_t N;
    int nlev;
    Dims ld[MAXLEV];
    double lh[MAXLEV];
    double *chain[MAXLEV][3];   // FP64 face coefficients per level; chain[0] = the fine copy
    // chain[0] not written by the last density load (the mixed modes' solve
    // forms the fine coefficients from rho); ensure_b64 forms it on demand
    bool b64_stale = false;
    // prolongation weights (one packed word per cell) of every level but the
    // coarsest, formed from the chain: shared by both hierarchies
    unsigned *pw[MAXLEV];
    // general operator A - diag(sigma) (pp_setup_general): closed links
    // allowed; sigma per level in FP64 (coarse sigma = mean of the 8
    // children); the active cells of level 0 and their count
    bool gen;
    bool sig_on;                 // sigma arrays exist
    bool singular;               // sigma is 0 everywhere: constants on the active cells are the null space
    double *sig[MAXLEV];
    unsigned char *act;
    double nact;
    // the cell densities of the last pp_update_density (allocated by its first
    // call); rho_ok while the fine coefficients are the ones formed from them,
    // so the outer operator kernels may form them again instead of reading
    // the three coefficient arrays
    double *rho;
    bool rho_ok;
    Hier hmix;                   // FP32 / FP16 hierarchy (mixed precision)
    Hier h64;                    // FP64 hierarchy (FP64 mode, and the mixed-mode fallback)
    double *pinv;
    int ncoarse;
    double *hcoarse;             // pinned: the coarsest level's beta (3 arrays) and sigma, read back
    double *hiter;               // pinned: the scalars of the last two outer iterations, read back
                                 // (HSLOT doubles each: the S_NSLOTS values, then a ticket)
    double ticket;               // the last ticket handed to a publishing kernel
    double iter_ticket[2];       // the ticket of each hiter slot's pending publication
    double scal_ticket;          // ... and of hscal's
    bool dot_on;                 // set by the outer loop: the fine-level pass that finishes the
    int dot_np;                  // V-cycle also forms the partials of r . z (dot_np of them,
                                 // r the V-cycle's scaled right-hand side)
    hipEvent_t iter_ev[2];       // their copies done
    hipEvent_t scal_ev;          // the scalar block's read-back (hscal) done
    hipEvent_t coarse_ev;        // the coarsest coefficients' read-back (hcoarse) done
    double *hpinv;               // pinned: the pseudo-inverse on its way to pinv
    hipStream_t copy_stream;     // its upload, beside the stream's work ...
    hipEvent_t pinv_ev;          // ... done
    hipEvent_t pinv_free;        // recorded where no V-cycle that reads pinv is still
    bool pinv_free_set;          // queued after it: the upload need wait for nothing later
    hipStream_t aux_stream;      // pp_step's divergence and cold-start residual, beside the
    hipEvent_t aux_start;        // coefficient load: the stream's earlier work done (u*
    hipEvent_t aux_done;         // written) ... and that side-stream work done
    bool pinv_wait;              // the next V-cycle waits for the upload before its coarse levels
    bool pinv_dirty;             // the coefficients changed since pinv was built: the next
                                 // V-cycle's caller builds it first (from hcoarse)
    bool check_pending;          // a density load's validity counts still to be read back
                                 // (by the next solve's first wait): pp_step
    bool scale_queued;           // the first V-cycle's scaled right-hand side is already queued
    bool init_queued;            // pp_step queued the cold start's initial residual (rows 3..5
    bool init_scaled;            // of part) and, for PCG, its scaling, on aux_stream
    bool check_rho_count;        // ... including the separate density count (S_SBAD)
    double *r64, *d64, *d64b, *q64;
    double *part;
    size_t pstride;
    double *scal;
    double *hscal;
    std::vector<void *> allocs;
    int64_t bytes;
    // kernel timing
    bool timing;
    uint32_t timing_mask;     // bit k: time launches of kind k
    std::vector<EventPair> ev;
    size_t ev_used;
    int64_t kt_count[PP_KT_COUNT];
    double kt_ms[PP_KT_COUNT];
};

namespace {

int dev_alloc(pp_ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0)
        bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(PP_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                   hipGetErrorString(e));
    }
    c->allocs.push_back(*p);
    c->bytes += (int64_t)bytes;
    return PP_OK;
}

template <typename P>
int dev_alloc_t(pp_ctx *c, P **p, size_t bytes)
{
    void *v = nullptr;
    int rc = dev_alloc(c, &v, bytes);
    *p = static_cast<P *>(v);
    return rc;
}

Dims to_dims(const pp_grid *g) { return Dims{g->n[0], g->n[1], g->n[2]}; }
Bc to_bc(const pp_grid *g) { return Bc{g->bc[0] == PP_WALL, g->bc[1] == PP_WALL, g->bc[2] == PP_WALL}; }

int validate_grid(const pp_grid *g, int *nlev_out, Dims *ld, double *lh, int coarsest = 64)
{
    if (!g)
        return fail(PP_EINVAL, "grid is NULL");
    for (int m = 0; m < 3; ++m) {
        if (g->n[m] < 4)
            return fail(PP_EINVAL, "grid: every n[m] must be >= 4 (got " + std::to_string(g->n[m]) + ")");
        if (g->n[m] > (1 << 16))
            return fail(PP_EINVAL, "grid: n[m] must be <= 65536");
        if (g->bc[m] != PP_PERIODIC && g->bc[m] != PP_WALL)
            return fail(PP_EINVAL, "grid: bc[m] must be PP_PERIODIC or PP_WALL");
    }
    if (!(g->h > 0.0) || !std::isfinite(g->h))
        return fail(PP_EINVAL, "grid: h must be a finite positive number");
    const double ncell = (double)g->n[0] * g->n[1] * g->n[2];
    if (ncell > 4.0e9)
        return fail(PP_EINVAL, "grid: more than 4e9 cells");
    if (nlev_out) {
        Dims d = to_dims(g);
        double h = g->h;
        int l = 0;
        ld[0] = d;
        lh[0] = h;
        while (d.nx % 2 == 0 && d.ny % 2 == 0 && d.nz % 2 == 0 && d.nx >= 8 && d.ny >= 8 &&
               d.nz >= 8 && cells(d) > (size_t)coarsest && l + 1 < MAXLEV) {
            d = Dims{d.nx / 2, d.ny / 2, d.nz / 2};
            h *= 2.0;
            ++l;
            ld[l] = d;
            lh[l] = h;
        }
        if (cells(d) > (size_t)COARSEST_MAX)
            return fail(PP_EINVAL, "grid: halving all directions while every n is even and >= 8 stops at " +
                                       std::to_string(d.nx) + "x" + std::to_string(d.ny) + "x" +
                                       std::to_string(d.nz) + " cells (> 1024)");
        *nlev_out = l + 1;
    }
    return PP_OK;
}

// the smoother's over-relaxation: red-black SOR converges for 0 < omega < 2
bool omega_ok(double omega) { return omega > 0.0 && omega < 2.0; }

int validate_opts(const pp_opts *o)
{
    if (o->precision < PP_FP64 || o->precision > PP_MIXED_FP16)
        return fail(PP_EINVAL, "opts.precision must be PP_FP64, PP_MIXED_FP32 or PP_MIXED_FP16");
    if (o->outer != PP_OUTER_PCG && o->outer != PP_OUTER_DC)
        return fail(PP_EINVAL, "opts.outer must be PP_OUTER_PCG or PP_OUTER_DC");
    if (o->nu_pre < 1 || o->nu_pre > 16 || o->nu_post < 1 || o->nu_post > 16)
        return fail(PP_EINVAL, "opts.nu_pre / nu_post must be in 1..16");
    if (o->max_outer < 1 || o->max_outer > 4096)
        return fail(PP_EINVAL, "opts.max_outer must be in 1..4096");
    if (o->warm_start != 0 && o->warm_start != 1)
        return fail(PP_EINVAL, "opts.warm_start must be 0 or 1");
    if (o->fallback != 0 && o->fallback != 1)
        return fail(PP_EINVAL, "opts.fallback must be 0 or 1");
    if (o->coarse_graph != 0 && o->coarse_graph != 1)
        return fail(PP_EINVAL, "opts.coarse_graph must be 0 or 1");
    if (o->nu_coarse < 1 || o->nu_coarse > 16)
        return fail(PP_EINVAL, "opts.nu_coarse must be in 1..16");
    if (!omega_ok(o->omega))
        return fail(PP_EINVAL, "opts.omega must be in (0, 2)");
    if (o->cycle != PP_CYCLE_V && o->cycle != PP_CYCLE_W && o->cycle != PP_CYCLE_F)
        return fail(PP_EINVAL, "opts.cycle must be PP_CYCLE_V, PP_CYCLE_W or PP_CYCLE_F");
    if (o->coarsest < 1 || o->coarsest > COARSEST_MAX)
        return fail(PP_EINVAL, "opts.coarsest must be in 1..1024");
    return PP_OK;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------

void resolve_timing(pp_ctx *c);

// Times the one kernel launched in its scope: the event pair goes to that
// launch (PP_LAUNCH), which takes the kernel's own start and end; a scope whose
// launch did not take them leaves its slot unused.
struct KT {
    pp_ctx *c;
    size_t slot;
    KT(pp_ctx *ctx, int k, bool fine) : c(ctx), slot((size_t)-1)
    {
        if (!c->timing || !fine || !((c->timing_mask >> k) & 1u))
            return;
        if (c->ev_used >= c->ev.size())
            resolve_timing(c);   // waits for the stream, then reuses the pool
        if (c->ev_used >= c->ev.size())
            return;
        slot = c->ev_used++;
        c->ev[slot].kind = k;
        g_launch_timer = LaunchTimer{c->ev[slot].a, c->ev[slot].b};
    }
    ~KT()
    {
        if (slot == (size_t)-1)
            return;
        if (g_launch_timer.start == c->ev[slot].a) {
            g_launch_timer = LaunchTimer{};
            c->ev[slot].kind = -1;
        }
    }
};

void resolve_timing(pp_ctx *c)
{
    if (c->ev_used == 0)
        return;
    (void)hipStreamSynchronize(c->stream);
    for (size_t i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        if (c->ev[i].kind >= 0 &&
            hipEventElapsedTime(&ms, c->ev[i].a, c->ev[i].b) == hipSuccess) {
            c->kt_ms[c->ev[i].kind] += ms;
            c->kt_count[c->ev[i].kind] += 1;
        }
    }
    c->ev_used = 0;
}

// ---------------------------------------------------------------------------
// hierarchy
// ---------------------------------------------------------------------------

int alloc_hier(pp_ctx *c, Hier &H, int st)
{
    H.st = st;
    H.nlev = c->nlev;
    H.present = true;
    H.tail = c->nlev - 1;
    while (H.tail > 0 && cells(c->ld[H.tail - 1]) <= TAIL_CELLS && c->nlev - (H.tail - 1) <= TAIL_MAX)
        --H.tail;
    const size_t sb = storage_bytes(st);
    for (int l = 0; l < c->nlev; ++l) {
        LevelBuf &v = H.lev[l];
        v.d = c->ld[l];
        v.h = c->lh[l];
        const size_t n = cells(v.d);
        for (int m = 0; m < 3; ++m) {
            if (st == ST_F64)
                v.b[m] = c->chain[l][m];
            else
                PP_TRY(dev_alloc(c, &v.b[m], n * sb));
        }
        PP_TRY(dev_alloc(c, &v.e, n * sb));
        PP_TRY(dev_alloc(c, &v.e2, n * sb));
        PP_TRY(dev_alloc(c, &v.r, n * sb));
        v.s = nullptr;
        if (c->sig_on)          // h^2 sigma of the level, in the storage type
            PP_TRY(dev_alloc(c, &v.s, n * sb));
        v.cur = v.e;
    }
    return PP_OK;
}

int read_scal(pp_ctx *c);

int fill_hier(pp_ctx *c, Hier &H, int from)
{
    if (!H.present)
        return PP_OK;
    if (H.st != ST_F64) {
        for (int l = from; l < c->nlev; ++l) {
            const size_t n = cells(c->ld[l]);
            for (int m = 0; m < 3; ++m) {
                if (H.st == ST_F32)
                    launch_convert<float>(n, c->chain[l][m], (float *)H.lev[l].b[m], c->stream);
                else
                    launch_convert<_Float16>(n, c->chain[l][m], (_Float16 *)H.lev[l].b[m], c->stream);
            }
        }
    }
    if (c->sig_on) {
        // the V-cycle keeps h^2 sigma: the unit of the face coefficients in the
        // smoother; FP16 storage must hold it (|h^2 sigma| < 6e4)
        const double limit = H.st == ST_F16 ? 6.0e4 : (H.st == ST_F32 ? 1.0e38 : INFINITY);
        const int maxb = (int)(2 * c->pstride);
        for (int l = 0; l < c->nlev; ++l) {
            const size_t n = cells(c->ld[l]);
            const double h2 = c->lh[l] * c->lh[l];
            int np;
            if (H.st == ST_F64)
                np = launch_convert_scaled<double>(n, c->sig[l], h2, limit, (double *)H.lev[l].s,
                                                   c->part, maxb, c->stream);
            else if (H.st == ST_F32)
                np = launch_convert_scaled<float>(n, c->sig[l], h2, limit, (float *)H.lev[l].s,
                                                  c->part, maxb, c->stream);
            else
                np = launch_convert_scaled<_Float16>(n, c->sig[l], h2, limit, (_Float16 *)H.lev[l].s,
                                                     c->part, maxb, c->stream);
            launch_finalize(c->part, c->pstride, np, OP_STORE, S_COUNT, (double)n, 0, c->scal,
                            c->stream);
            PP_TRY(read_scal(c));
            if (c->hscal[S_COUNT] != 0.0)
                return fail(PP_EINVAL, "sigma: h^2 sigma of level " + std::to_string(l) +
                                           " does not fit the storage precision (use FP32 or FP64)");
        }
    }
    return check_launch("convert coefficients");
}

// In place, lower triangle (row-major), right-looking: after column j is
// scaled, every entry of the trailing lower triangle takes its update
// independently (row by row over contiguous memory), so the loops carry no
// chain of dependent additions.  The pseudo-inverse is rebuilt on the host
// at every coefficient update, overlapping the GPU's work before the first
// V-cycle needs it.
int cholesky(std::vector<double> &a, int n)
{
    std::vector<double> col((size_t)n);
    for (int j = 0; j < n; ++j) {
        const double dgl = a[(size_t)j * n + j];
        if (!(dgl > 0.0))
            return -1;
        const double d = std::sqrt(dgl);
        a[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            a[(size_t)i * n + j] /= d;
            col[i] = a[(size_t)i * n + j];
        }
        for (int i = j + 1; i < n; ++i) {
            const double lij = col[i];
            double *ai = &a[(size_t)i * n];
            for (int k = j + 1; k <= i; ++k)
                ai[k] -= lij * col[k];
        }
    }
    return 0;
}

// Enqueue the read-back of the coarsest level's coefficients into pinned
// host memory; build_pinv waits for it (coarse_ev) before reading them.
int enqueue_coarse_download(pp_ctx *c)
{
    const int L = c->nlev - 1;
    const size_t n = cells(c->ld[L]);
    const double *src[4] = {c->chain[L][0], c->chain[L][1], c->chain[L][2],
                            c->sig_on ? c->sig[L] : nullptr};
    launch_publish_arrays(src, c->sig_on ? 4 : 3, (int)n, c->hcoarse, c->stream);
    PP_TRY(check_launch("coarsest coefficients read-back"));
    PP_HIP(hipEventRecord(c->coarse_ev, c->stream));
    return PP_OK;
}

// FP64 pseudo-inverse of the coarsest operator.  The pressure operator A is
// singular (constants in the null space): with K = -A + (s/n) 1 1^T positive
// definite, A^+ = (1/(s n)) 1 1^T - K^-1.  For the general operator
// A - diag(sigma) the same is done on the active coarse cells (a nonzero
// diagonal); when sigma is present the operator is definite there and
// A^+ = -K^-1 with K = -A + diag(sigma).  Excluded cells get zero rows and
// columns.
// The coarsest coefficients come from the pinned read-back of
// enqueue_coarse_download.
int build_pinv(pp_ctx *c)
{
    const int L = c->nlev - 1;
    const Dims d = c->ld[L];
    const int n = (int)cells(d);
    const double h = c->lh[L];
    const double *b[3] = {c->hcoarse, c->hcoarse + n, c->hcoarse + 2 * (size_t)n};
    const double *sg = c->sig_on ? c->hcoarse + 3 * (size_t)n : nullptr;
    std::vector<double> A((size_t)n * n, 0.0);
    const int nn[3] = {d.nx, d.ny, d.nz};
    const int wall[3] = {c->bc.x, c->bc.y, c->bc.z};
    for (int k = 0; k < d.nz; ++k)
        for (int j = 0; j < d.ny; ++j)
            for (int i = 0; i < d.nx; ++i) {
                const int R = (k * d.ny + j) * d.nx + i;
                int q[3] = {i, j, k};
                for (int m = 0; m < 3; ++m) {
                    int lo[3] = {q[0], q[1], q[2]};
                    lo[m] -= 1;
                    if (lo[m] < 0) {
                        if (wall[m])
                            continue;
                        lo[m] += nn[m];
                    }
                    const int Lc = (lo[2] * d.ny + lo[1]) * d.nx + lo[0];
                    const double w = b[m][R] / (h * h);
                    A[(size_t)R * n + R] -= w;
                    A[(size_t)R * n + Lc] += w;
                    A[(size_t)Lc * n + Lc] -= w;
                    A[(size_t)Lc * n + R] += w;
                }
                if (sg)
                    A[(size_t)R * n + R] -= sg[R];
            }
    std::vector<int> idx;
    for (int i = 0; i < n; ++i)
        if (A[(size_t)i * n + i] < 0.0)
            idx.push_back(i);
    const int na = (int)idx.size();
    if (na == 0)
        return fail(PP_EINVAL, "coarsest operator is zero");
    const bool singular = !c->gen || c->singular;
    double s = 0.0;
    for (int i = 0; i < na; ++i)
        s = std::max(s, -A[(size_t)idx[i] * n + idx[i]]);
    std::vector<double> K((size_t)na * na);
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < na; ++j)
            K[(size_t)i * na + j] = -A[(size_t)idx[i] * n + idx[j]] + (singular ? s / na : 0.0);
    if (cholesky(K, na) != 0)
        return fail(PP_EINVAL, "coarsest operator is not definite on mean-zero fields "
                               "(disconnected domain?)");
    // K^-1 = L^-T L^-1 = M^T M with M = L^-1, lower triangular.  M comes from
    // L M = I by forward substitution, all columns at once: row i of M is
    // (e_i - sum_{k<i} L_ik M_k) / L_ii over rows k already formed, each step
    // an update of a contiguous row.  M^T M is summed as outer products of
    // the rows of M.  No loop carries a chain of dependent additions.
    std::vector<double> M((size_t)na * na, 0.0);
    for (int i = 0; i < na; ++i) {
        double *mi = &M[(size_t)i * na];
        const double *li = &K[(size_t)i * na];
        mi[i] = 1.0;
        for (int k = 0; k < i; ++k) {
            const double lik = li[k];
            const double *mk = &M[(size_t)k * na];
            for (int q = 0; q <= k; ++q)
                mi[q] -= lik * mk[q];
        }
        const double inv = 1.0 / li[i];
        for (int q = 0; q <= i; ++q)
            mi[q] *= inv;
    }
    std::vector<double> G((size_t)na * na, 0.0);   // M^T M, lower triangle
    for (int k = 0; k < na; ++k) {
        const double *mk = &M[(size_t)k * na];
        for (int a = 0; a <= k; ++a) {
            const double mka = mk[a];
            double *ga = &G[(size_t)a * na];
            for (int bb = 0; bb <= a; ++bb)
                ga[bb] += mka * mk[bb];
        }
    }
    // the previous upload has read hpinv (it completed before that solve's
    // coarse levels ran, so this returns at once)
    PP_HIP(hipEventSynchronize(c->pinv_ev));
    double *P = c->hpinv;
    std::fill(P, P + (size_t)n * n, 0.0);
    const double shift = singular ? 1.0 / (s * na) : 0.0;
    for (int a = 0; a < na; ++a)
        for (int bb = 0; bb <= a; ++bb) {
            const double v = shift - G[(size_t)a * na + bb];
            P[(size_t)idx[a] * n + idx[bb]] = v;
            P[(size_t)idx[bb] * n + idx[a]] = v;
        }
    // The upload goes on a stream of its own, behind everything queued so far
    // (no earlier coarsest solve can still read pinv), or only behind
    // pinv_free where that was recorded, so the work the host queues next, up
    // to the first coarse level, does not wait for the copy; that V-cycle
    // waits for it before its coarse levels (pinv_wait)
    if (c->pinv_free_set) {
        PP_HIP(hipStreamWaitEvent(c->copy_stream, c->pinv_free, 0));
        c->pinv_free_set = false;
    } else {
        PP_HIP(hipEventRecord(c->pinv_ev, c->stream));
        PP_HIP(hipStreamWaitEvent(c->copy_stream, c->pinv_ev, 0));
    }
    PP_HIP(hipMemcpyAsync(c->pinv, P, sizeof(double) * n * n, hipMemcpyHostToDevice,
                          c->copy_stream));
    PP_HIP(hipEventRecord(c->pinv_ev, c->copy_stream));
    c->pinv_wait = true;
    return PP_OK;
}

// Wait until the kernel queued before `ev` has written `ticket` to *flag, in
// pinned, coherent host memory, after the values it publishes.  Polling the
// flag sees them as soon as the kernel has written them, before the end of the
// kernel reaches the host as an event.  The event bounds the wait: once it has
// completed, the flag holds the ticket (the kernel fences its writes first).
int wait_ticket(const double *flag, double ticket, hipEvent_t ev)
{
    const volatile double *f = flag;
    for (unsigned n = 1; *f != ticket; ++n) {
        if ((n & 255u) == 0) {
            const hipError_t q = hipEventQuery(ev);
            if (q == hipSuccess) {
                if (*f == ticket)
                    break;
                return fail(PP_EHIP, "scalar read-back: the kernel ended without its ticket");
            }
            if (q != hipErrorNotReady)
                return fail(PP_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
        }
        _mm_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return PP_OK;
}

// the scalar block into hscal: post_scal queues the copy, wait_scal waits
// for it (host work in between overlaps the GPU's queue)
int post_scal(pp_ctx *c)
{
    c->scal_ticket = ++c->ticket;
    launch_publish(c->scal, c->hscal, S_NSLOTS, c->stream, c->scal_ticket);
    PP_TRY(check_launch("scalar read-back"));
    PP_HIP(hipEventRecord(c->scal_ev, c->stream));
    return PP_OK;
}

int wait_scal(pp_ctx *c)
{
    return wait_ticket(c->hscal + S_NSLOTS, c->scal_ticket, c->scal_ev);
}

int read_scal(pp_ctx *c)
{
    PP_TRY(post_scal(c));
    return wait_scal(c);
}

int nparts(pp_ctx *c) { return (int)grid_blocks(red_grid(c->d)); }

// the coarsest level's pseudo-inverse for the current coefficients, built on
// the host from the read-back coarsest coefficients and queued for upload
int ensure_pinv(pp_ctx *c)
{
    if (!c->pinv_dirty)
        return PP_OK;
    // the read-back of the coarsest coefficients (a load that does not wait
    // for its validity counts has not waited for it either)
    PP_HIP(hipEventSynchronize(c->coarse_ev));
    PP_TRY(build_pinv(c));
    c->pinv_dirty = false;
    return PP_OK;
}

// the prolongation weights of the levels from `from` on (all but the
// coarsest), from the FP64 chain
int build_weights(pp_ctx *c, int from)
{
    for (int l = from; l + 1 < c->nlev; ++l)
        launch_prolong_weights(c->ld[l], c->bc, c->chain[l][0], c->chain[l][1], c->chain[l][2],
                               c->pw[l], c->stream);
    return check_launch("prolongation weights");
}

// General operator: copy and check beta (closed links allowed) and sigma,
// mark the active cells, coarsen both through the levels, fill the storage
// hierarchies and build the coarsest pseudo-inverse.
int load_coeffs_general(pp_ctx *c, const double *bx, const double *by, const double *bz,
                        const double *sg)
{
    const double *src[3] = {bx, by, bz};
    for (int m = 0; m < 3; ++m)
        PP_HIP(hipMemcpyAsync(c->chain[0][m], src[m], sizeof(double) * c->N, hipMemcpyDeviceToDevice,
                              c->stream));
    launch_zero_walls(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2], c->stream);
    launch_check_beta(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2], true, c->part,
                      c->stream);
    launch_finalize(c->part, c->pstride, nparts(c), OP_STORE, S_COUNT, (double)c->N, 0, c->scal,
                    c->stream);
    if (c->sig_on) {
        PP_HIP(hipMemcpyAsync(c->sig[0], sg, sizeof(double) * c->N, hipMemcpyDeviceToDevice,
                              c->stream));
        launch_check_sigma(c->d, c->sig[0], c->part, c->pstride, c->stream);
        launch_finalize(c->part, c->pstride, nparts(c), OP_STORE, S_SBAD, (double)c->N, 0, c->scal,
                        c->stream);
        launch_finalize(c->part + c->pstride, c->pstride, nparts(c), OP_STORE, S_SPOS, (double)c->N,
                        0, c->scal, c->stream);
    }
    launch_active(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2],
                  c->sig_on ? c->sig[0] : nullptr, c->act, c->part, c->stream);
    launch_finalize(c->part, c->pstride, nparts(c), OP_STORE, S_NACT, (double)c->N, 0, c->scal,
                    c->stream);
    PP_TRY(check_launch("coefficient check"));
    for (int l = 0; l + 1 < c->nlev; ++l) {
        launch_coarsen_beta(c->ld[l], c->bc, c->chain[l][0], c->chain[l][1], c->chain[l][2],
                            c->chain[l + 1][0], c->chain[l + 1][1], c->chain[l + 1][2], c->stream);
        if (c->sig_on)
            launch_coarsen_sigma(c->ld[l], c->sig[l], c->sig[l + 1], c->stream);
    }
    PP_TRY(check_launch("coarsen coefficients"));
    PP_TRY(build_weights(c, 0));
    PP_TRY(read_scal(c));
    if (c->hscal[S_COUNT] != 0.0)
        return fail(PP_EINVAL, "beta: " + std::to_string((long long)c->hscal[S_COUNT]) +
                                   " non-wall faces are not finite non-negative numbers");
    if (c->sig_on && c->hscal[S_SBAD] != 0.0)
        return fail(PP_EINVAL, "sigma: " + std::to_string((long long)c->hscal[S_SBAD]) +
                                   " entries are not finite non-negative numbers");
    PP_TRY(fill_hier(c, c->hmix, 0));
    PP_TRY(fill_hier(c, c->h64, 0));
    PP_TRY(enqueue_coarse_download(c));
    PP_TRY(read_scal(c));
    c->singular = !(c->sig_on && c->hscal[S_SPOS] > 0.0);
    c->nact = c->hscal[S_NACT];
    if (!(c->nact > 0.0))
        return fail(PP_EINVAL, "no cell has an open face or a diagonal term");
    c->pinv_dirty = true;
    return PP_OK;
}

// Level-0 coefficients into the FP64 chain (and the mixed hierarchy's level
// 0 and level 1 where the one-pass kernel applies), then the coarse levels,
// the storage copies and the coarsest pseudo-inverse.  The coefficients come
// from the caller's beta arrays, or (rho non-null) are computed from the
// cell densities.
// the verdict on a coefficient load from its validity counts, read back in
// hscal (rho: the coefficients came from densities; rho_count: the densities
// were counted by their own pass, into S_SBAD)
int coeff_verdict(pp_ctx *c, bool rho, bool rho_count)
{
    const double nbad = c->hscal[S_COUNT] + (rho_count ? c->hscal[S_SBAD] : 0.0);
    if (nbad == 0.0)
        return PP_OK;
    c->rho_ok = false;
    if (rho)
        return fail(PP_EINVAL, "rho: " + std::to_string((long long)nbad) +
                                   " cells or faces are not finite positive numbers "
                                   "(density, or the face coefficient 2 / (rho_L + rho_R))");
    return fail(PP_EINVAL, "beta: " + std::to_string((long long)c->hscal[S_COUNT]) +
                               " non-wall faces are not finite positive numbers");
}

// defer: leave the validity counts for the next solve's first wait (which
// reports a rejection) instead of waiting for them here
int load_coeffs_impl(pp_ctx *c, const double *const src[3], const double *rho, bool defer = false)
{
    c->rho_ok = false;
    c->check_pending = false;
    c->b64_stale = false;
    if (rho && !c->rho)
        PP_TRY(dev_alloc_t(c, &c->rho, sizeof(double) * c->N));
    int first_coarse = 0;   // first level whose coefficients are still to be coarsened from
    bool level0_converted = false;
    const uintptr_t align = rho ? (uintptr_t)rho
                                : ((uintptr_t)src[0] | (uintptr_t)src[1] | (uintptr_t)src[2]);
    bool rho_checked = false;
    if (c->nlev > 1 && !(align & 15)) {
        // one pass: copy (or beta from rho), walls, validity, storage copy of
        // level 0, level 1.  From densities in a mixed mode the FP64 fine
        // coefficients are left unwritten: the outer kernels form them from
        // the copy of rho, and ensure_b64 writes them for anything else.
        const Hier &H = c->hmix;
        const bool skip64 = rho && H.present && (H.st == ST_F32 || H.st == ST_F16);
        double *dst[3] = {c->chain[0][0], c->chain[0][1], c->chain[0][2]};
        if (skip64)
            dst[0] = dst[1] = dst[2] = nullptr;
        c->b64_stale = skip64;
        double *crs[3] = {c->chain[1][0], c->chain[1][1], c->chain[1][2]};
        int np = 0;
        auto one_pass = [&](auto *t) {
            using TT = std::remove_pointer_t<decltype(t)>;
            TT *tt[3] = {t, t ? (TT *)H.lev[0].b[1] : nullptr, t ? (TT *)H.lev[0].b[2] : nullptr};
            return rho ? launch_load_density<TT>(c->d, c->bc, rho, dst, tt, crs, c->rho, c->pw[0],
                                                 c->part, c->stream)
                       : launch_load_coeffs<TT>(c->d, c->bc, src, dst, tt, crs, c->pw[0], c->part,
                                                c->stream);
        };
        if (H.present && H.st == ST_F32) {
            np = one_pass((float *)H.lev[0].b[0]);
            level0_converted = true;
        } else if (H.present && H.st == ST_F16) {
            np = one_pass((_Float16 *)H.lev[0].b[0]);
            level0_converted = true;
        } else {
            np = one_pass((float *)nullptr);
        }
        launch_finalize(c->part, c->pstride, np, OP_STORE, S_COUNT, (double)c->N, 0, c->scal,
                        c->stream);
        first_coarse = 1;
        rho_checked = rho != nullptr;
    } else {
        if (rho) {
            launch_face_coeffs(c->d, c->bc, rho, c->chain[0][0], c->chain[0][1], c->chain[0][2],
                               c->stream);
            PP_HIP(hipMemcpyAsync(c->rho, rho, sizeof(double) * c->N, hipMemcpyDeviceToDevice,
                                  c->stream));
        } else {
            for (int m = 0; m < 3; ++m)
                PP_HIP(hipMemcpyAsync(c->chain[0][m], src[m], sizeof(double) * c->N,
                                      hipMemcpyDeviceToDevice, c->stream));
            launch_zero_walls(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2],
                              c->stream);
        }
        launch_check_beta(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2], false,
                          c->part, c->stream);
        launch_finalize(c->part, c->pstride, nparts(c), OP_STORE, S_COUNT, (double)c->N, 0,
                        c->scal, c->stream);
    }
    const bool rho_count = rho && !rho_checked;   // densities counted by their own pass
    if (rho_count) {
        launch_check_rho(c->d, rho, c->part, c->stream);
        launch_finalize(c->part, c->pstride, nparts(c), OP_STORE, S_SBAD, (double)c->N, 0,
                        c->scal, c->stream);
    }
    PP_TRY(check_launch("coefficient check"));
    int conv_from = level0_converted ? 1 : 0;
    if (first_coarse == 1 && level0_converted) {
        // every further level but the coarsest in one pass each, with the
        // kernel of level 0 reading the chain in place: the storage copy,
        // the prolongation weights and the next level's coefficients (their
        // validity count is not needed: coarse coefficients are positive
        // means of valid fine ones)
        const Hier &H = c->hmix;
        for (int l = 1; l + 1 < c->nlev; ++l) {
            double *lev[3] = {c->chain[l][0], c->chain[l][1], c->chain[l][2]};
            const double *src[3] = {lev[0], lev[1], lev[2]};
            double *crs[3] = {c->chain[l + 1][0], c->chain[l + 1][1], c->chain[l + 1][2]};
            // the last of them also writes the coarsest level's storage copy
            const bool last = l + 2 == c->nlev;
            auto go = [&](auto *t) {
                using TT = std::remove_pointer_t<decltype(t)>;
                TT *tt[3] = {(TT *)H.lev[l].b[0], (TT *)H.lev[l].b[1], (TT *)H.lev[l].b[2]};
                TT *ct[3] = {(TT *)H.lev[l + 1].b[0], (TT *)H.lev[l + 1].b[1],
                             (TT *)H.lev[l + 1].b[2]};
                launch_load_coeffs<TT>(c->ld[l], c->bc, src, lev, tt, crs, c->pw[l], nullptr,
                                       c->stream, last ? ct : nullptr);
            };
            if (H.st == ST_F32)
                go((float *)nullptr);
            else
                go((_Float16 *)nullptr);
        }
        // the coarsest level's storage copy is written above when there are
        // levels between it and level 0; otherwise it is level 1, converted
        conv_from = c->nlev > 2 ? c->nlev : 1;
    } else {
        for (int l = first_coarse; l + 1 < c->nlev; ++l)
            launch_coarsen_beta(c->ld[l], c->bc, c->chain[l][0], c->chain[l][1], c->chain[l][2],
                                c->chain[l + 1][0], c->chain[l + 1][1], c->chain[l + 1][2],
                                c->stream);
        PP_TRY(build_weights(c, first_coarse));   // the one-pass kernel formed level 0's
    }
    PP_TRY(check_launch("coarsen coefficients"));
    PP_TRY(fill_hier(c, c->hmix, conv_from));
    PP_TRY(enqueue_coarse_download(c));
    // the coarsest pseudo-inverse is built on the host by the next solve,
    // while the GPU works through what is queued before it
    c->pinv_dirty = true;
    c->rho_ok = rho != nullptr;
    if (defer) {
        c->check_pending = true;
        c->check_rho_count = rho_count;
        return PP_OK;
    }
    PP_TRY(read_scal(c));
    return coeff_verdict(c, rho != nullptr, rho_count);
}

int load_coeffs(pp_ctx *c, const double *bx, const double *by, const double *bz)
{
    const double *src[3] = {bx, by, bz};
    return load_coeffs_impl(c, src, nullptr);
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------

// nu out-of-place sweeps on a large level starting from the correction in
// cur (ignored when zero_first), ping-ponging between e and e2; returns the
// buffer holding the result.  FP32 and FP16 storage take two sweeps per pass
// where the level allows it (the second pass of an odd nu is a single sweep).
template <typename T>
void *fused_sweeps(pp_ctx *c, LevelBuf &v, int l, int nu, void *cur, int first_colour,
                   bool zero_first, hipStream_t s, bool dot = false)
{
    const double h2 = v.h * v.h;
    const T *b0 = (const T *)v.b[0], *b1 = (const T *)v.b[1], *b2 = (const T *)v.b[2];
    for (int sw = 0; sw < nu;) {
        void *out = (cur == v.e) ? v.e2 : v.e;
        KT t(c, PP_KT_SMOOTH, l == 0);
        const bool zero = zero_first && sw == 0;
        bool two = false;
        if constexpr (!std::is_same<T, double>::value) {
            if (sw + 2 <= nu && fused2_fits(v.d)) {
                // the last pass may also form the outer loop's dot product
                const bool last = sw + 2 == nu;
                const int np = launch_rbgs_fused2<T>(
                    v.d, c->bc, b0, b1, b2, (const T *)v.r, (const T *)cur, (T *)out,
                    (const T *)v.s, h2, c->opts.omega, first_colour, zero, s,
                    (last && dot) ? c->part : nullptr);
                if (last && np > 0)
                    c->dot_np = np;
                two = true;
            }
        }
        if (!two)
            launch_rbgs_fused<T>(v.d, c->bc, b0, b1, b2, (const T *)v.r, (const T *)cur, (T *)out,
                                 (const T *)v.s, h2, c->opts.omega, first_colour, zero, s);
        sw += two ? 2 : 1;
        cur = out;
    }
    return cur;
}

// nu_pre red-black sweeps (red first) from e = 0 on level l, then residual +
// restriction into the right-hand side of level l + 1.  Large levels use the
// fused out-of-place sweep (ping-pong between e and e2); smaller ones, where
// the fused kernel's march along z is latency-bound, use one launch per
// colour in place.  warm: the sweeps start from the level's current
// correction (the second coarse correction of a W-cycle).
template <typename T>
void level_down(pp_ctx *c, Hier &H, int l, hipStream_t s, bool warm = false)
{
    LevelBuf &v = H.lev[l];
    const double h2 = v.h * v.h;
    const T *b0 = (const T *)v.b[0], *b1 = (const T *)v.b[1], *b2 = (const T *)v.b[2];
    if (cells(v.d) > fused_min_cells<T>() && fused_plane_fits(v.d, sizeof(T))) {
        v.cur = warm ? fused_sweeps<T>(c, v, l, c->opts.nu_pre, v.cur, 0, false, s)
                     : fused_sweeps<T>(c, v, l, c->opts.nu_pre, v.e2, 0, true, s);
    } else {
        T *e = warm ? (T *)v.cur : (T *)v.e;
        for (int sw = 0; sw < c->opts.nu_pre; ++sw) {
            const bool z = !warm && sw == 0;
            launch_rbgs<T>(v.d, c->bc, b0, b1, b2, (const T *)v.r, e, (const T *)v.s, h2,
                           c->opts.omega, 0, z, false, s);
            launch_rbgs<T>(v.d, c->bc, b0, b1, b2, (const T *)v.r, e, (const T *)v.s, h2,
                           c->opts.omega, 1, false, z, s);
        }
        v.cur = e;
    }
    KT t(c, PP_KT_RESTRICT, l == 0);
    launch_resid_restrict<T>(v.d, c->bc, b0, b1, b2, (const T *)v.cur, (const T *)v.r,
                             (const T *)v.s, (T *)H.lev[l + 1].r, 1.0 / h2, s);
}

// prolongation + correction from level l + 1, then nu_post sweeps (black
// first): the mirror image of level_down, so the cycle is symmetric
template <typename T>
void level_up(pp_ctx *c, Hier &H, int l, hipStream_t s)
{
    LevelBuf &v = H.lev[l];
    const double h2 = v.h * v.h;
    const T *b0 = (const T *)v.b[0], *b1 = (const T *)v.b[1], *b2 = (const T *)v.b[2];
    {
        KT t(c, PP_KT_PROLONG, l == 0);
        launch_prolong<T>(v.d, c->bc, (const T *)H.lev[l + 1].cur, (T *)v.cur, c->pw[l], s);
    }
    if (cells(v.d) > fused_min_cells<T>() && fused_plane_fits(v.d, sizeof(T))) {
        v.cur = fused_sweeps<T>(c, v, l, c->opts.nu_post, v.cur, 1, false, s,
                                l == 0 && c->dot_on);
    } else {
        for (int sw = 0; sw < c->opts.nu_post; ++sw) {
            launch_rbgs<T>(v.d, c->bc, b0, b1, b2, (const T *)v.r, (T *)v.cur, (const T *)v.s, h2,
                           c->opts.omega, 1, false, false, s);
            launch_rbgs<T>(v.d, c->bc, b0, b1, b2, (const T *)v.r, (T *)v.cur, (const T *)v.s, h2,
                           c->opts.omega, 0, false, false, s);
        }
    }
}

// levels t .. L-1 (the tail) in one single-workgroup kernel, in place on e
template <typename T>
void run_tail(pp_ctx *c, Hier &H, int t, hipStream_t s, bool warm = false)
{
    const int n = H.nlev - t;
    Dims d[TAIL_MAX];
    double h2[TAIL_MAX];
    const void *b[TAIL_MAX][3];
    void *e[TAIL_MAX];
    void *r[TAIL_MAX];
    const void *sg[TAIL_MAX];
    const unsigned *w[TAIL_MAX];
    for (int q = 0; q < n; ++q) {
        LevelBuf &v = H.lev[t + q];
        w[q] = c->pw[t + q];
        d[q] = v.d;
        h2[q] = v.h * v.h;
        for (int m = 0; m < 3; ++m)
            b[q][m] = v.b[m];
        e[q] = v.e;
        r[q] = v.r;
        sg[q] = v.s;
        v.cur = v.e;
    }
    launch_tail<T>(n, d, h2, b, e, r, sg, w, c->bc, c->opts.nu_coarse, c->opts.nu_coarse,
                   c->opts.omega, c->pinv, c->ncoarse, warm, s);
}

// The cycle on levels l .. L-1 for A e = r (input lev[l].r, output
// lev[l].cur); warm: level l starts from its current correction.  Each level
// above the tail takes its coarse correction once (V), or twice, the second
// pass starting from the correction the first one left on the next level: by
// the same cycle (W) or by a V-cycle (F).
template <typename T>
void cycle_level(pp_ctx *c, Hier &H, int l, bool warm, int kind, hipStream_t s)
{
    if (l >= H.tail) {
        run_tail<T>(c, H, l, s, warm);
        return;
    }
    level_down<T>(c, H, l, s, warm);
    cycle_level<T>(c, H, l + 1, false, kind, s);
    if (kind != PP_CYCLE_V)
        cycle_level<T>(c, H, l + 1, true, kind == PP_CYCLE_W ? PP_CYCLE_W : PP_CYCLE_V, s);
    level_up<T>(c, H, l, s);
}

// the coarse correction of level from - 1: the cycle on levels from .. L-1
// (input: lev[from].r), once or, for W- and F-cycles, twice
template <typename T>
void cycle_from(pp_ctx *c, Hier &H, int from, hipStream_t s)
{
    const int kind = c->opts.cycle;
    cycle_level<T>(c, H, from, false, kind, s);
    if (kind != PP_CYCLE_V && from > 0)
        cycle_level<T>(c, H, from, true, kind == PP_CYCLE_W ? PP_CYCLE_W : PP_CYCLE_V, s);
}

// One V-cycle for A e = r on level 0 (input lev[0].r, output lev[0].cur).
// Levels 1 .. L-1 are short kernels whose cost is launch latency; they are
// replayed from a HIP graph captured at setup when one is available.
template <typename T>
int vcycle_run(pp_ctx *c, Hier &H)
{
    hipStream_t s = c->stream;
    // a pseudo-inverse still to be built (pp_step leaves it to the first
    // V-cycle, whose fine-level pass the GPU works on meanwhile) or an upload
    // still on its way: the coarse levels wait for it
    auto await_pinv = [c, s]() -> int {
        PP_TRY(ensure_pinv(c));
        if (c->pinv_wait) {
            (void)hipStreamWaitEvent(s, c->pinv_ev, 0);
            c->pinv_wait = false;
        }
        return PP_OK;
    };
    if (H.tail == 0) {
        PP_TRY(await_pinv());
        cycle_from<T>(c, H, 0, s);
        return PP_OK;
    }
    level_down<T>(c, H, 0, s);
    PP_TRY(await_pinv());
    if (!H.coarse_exec || hipGraphLaunch(H.coarse_exec, s) != hipSuccess)
        cycle_from<T>(c, H, 1, s);    // no graph, or it could not be launched: run eagerly
    level_up<T>(c, H, 0, s);
    return PP_OK;
}

// Record levels 1 .. L-1 of the cycle into a graph on a private stream.  The
// host-side bookkeeping of which correction buffer is current is the same at
// every replay, because the captured sequence is fixed.
template <typename T>
int capture_coarse(pp_ctx *c, Hier &H)
{
    if (!H.present || H.tail < 2)
        return PP_OK;             // levels 1 .. L-1 are one kernel or none
    prepare_fused<T>();
    if constexpr (!std::is_same<T, double>::value)
        prepare_fused2<T>();
    hipStream_t cap = nullptr;
    PP_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        cycle_from<T>(c, H, 1, cap);
        e = hipStreamEndCapture(cap, &g);
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&H.coarse_exec, g, nullptr, nullptr, 0);
    if (g)
        (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        H.coarse_exec = nullptr;
        return fail(PP_EHIP, std::string("capturing the coarse-level graph: ") + hipGetErrorString(e));
    }
    return PP_OK;
}

int capture_graphs(pp_ctx *c)
{
    if (!c->opts.coarse_graph)
        return PP_OK;
    for (Hier *H : {&c->hmix, &c->h64}) {
        if (!H->present)
            continue;
        int rc = PP_OK;
        switch (H->st) {
        case ST_F64: rc = capture_coarse<double>(c, *H); break;
        case ST_F32: rc = capture_coarse<float>(c, *H); break;
        default: rc = capture_coarse<_Float16>(c, *H); break;
        }
        if (rc != PP_OK)
            return rc;
    }
    return PP_OK;
}

// ---------------------------------------------------------------------------
// outer iterations
// ---------------------------------------------------------------------------

struct SolveState {
    double nb;
    double rel;
    double best;
    int it;
    pp_stats *st;
};

void record(SolveState &S)
{
    if (S.st && S.it >= 1 && S.it <= PP_HIST)
        S.st->res_hist[S.it - 1] = S.rel;
}

int check_progress(SolveState &S, int since_best_limit, int &since, double &best_window)
{
    if (!std::isfinite(S.rel))
        return fail(PP_EDIVERGED, "residual is not finite");
    if (S.rel > 1e3 * S.best)
        return fail(PP_EDIVERGED, "residual grew a thousandfold above its best value");
    S.best = std::min(S.best, S.rel);
    if (S.rel < 0.9 * best_window) {
        best_window = S.rel;
        since = 0;
    } else if (++since >= since_best_limit) {
        return STAGNATED;
    }
    return PP_OK;
}

// the densities the fine coefficients were formed from, or null: the outer
// operator kernels then read the coefficient arrays
const double *op_rho(const pp_ctx *c) { return (c->rho_ok && !c->gen) ? c->rho : nullptr; }

// the FP64 fine-level coefficients for a reader that takes them from chain[0]
// (pp_apply, defect correction, the FP64 fallback, and the outer kernels
// before a density load is confirmed): formed from the context's copy of rho
// by the expression the density load uses, so with the same bits
int ensure_b64(pp_ctx *c)
{
    if (!c->b64_stale)
        return PP_OK;
    launch_face_coeffs(c->d, c->bc, c->rho, c->chain[0][0], c->chain[0][1], c->chain[0][2],
                       c->stream);
    c->b64_stale = false;
    return check_launch("fine-level coefficients from rho");
}

int gauge(pp_ctx *c, double *x, int xsum_parts = 0);

// work a caller queues behind a solve's result (the projection of pp_step)
using Tail = std::function<int()>;

// residual of the current iterate into r64 (+ RR, BB, scales); returns rel.
// gauge_x: the gauge of x is queued behind the residual, before the host
// waits for it; it changes neither A x nor the residual (it removes a
// constant of the null space, or clears excluded cells, which no link
// reaches), so the iterate may go on from there.  tail (with gauge_x): queued
// behind the read-back, so the GPU has it to work on while the host waits; if
// the iterate goes on, it is queued again at the next confirmation.
int true_residual(pp_ctx *c, const double *rhs, double *x, bool zero_x, SolveState &S,
                  bool gauge_x = false, const Tail *tail = nullptr, const Tail *pre = nullptr)
{
    const double ih2 = 1.0 / (c->grid.h * c->grid.h);
    // a cold start's residual that pp_step queued already (b - mean b)
    const bool init_queued = zero_x && c->init_queued;
    c->init_queued = false;
    int np = 0;
    if (!init_queued) {
        if (!zero_x && !residual_from_rho(c->d, op_rho(c), rhs, x, c->r64))
            PP_TRY(ensure_b64(c));
        np = launch_residual(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2],
                             op_rho(c), rhs, c->scal, x, zero_x, c->sig_on ? c->sig[0] : nullptr,
                             c->gen ? c->act : nullptr, c->r64, ih2, c->part, c->pstride,
                             c->stream);
        launch_finalize(c->part, c->pstride, np, OP_INIT, 0, (double)c->N, 0, c->scal,
                        c->stream);
        PP_TRY(check_launch("residual"));
    }
    if (gauge_x)
        PP_TRY(gauge(c, x, zero_x ? 0 : np));   // the residual kernel summed x too
    PP_TRY(post_scal(c));
    if (gauge_x && tail)
        PP_TRY((*tail)());
    if (init_queued && c->init_scaled)
        c->scale_queued = true;      // queued with the residual
    else if (pre)
        PP_TRY((*pre)());
    c->init_scaled = false;
    // a pseudo-inverse still to be built is built here, on the host, while
    // the GPU works through the residual and whatever was queued before it;
    // its upload follows the read-back in the queue, unwaited.  After pp_step
    // queued the residual early, the GPU has little left before it: the first
    // V-cycle builds it instead, behind its first fine-level pass.
    if (init_queued && c->pinv_dirty) {
        // no V-cycle of this solve is queued yet, and every later one builds
        // the pseudo-inverse before reading it: its upload may start from here
        PP_HIP(hipEventRecord(c->pinv_free, c->stream));
        c->pinv_free_set = true;
    }
    const int prc = init_queued ? PP_OK : ensure_pinv(c);
    PP_TRY(wait_scal(c));
    if (c->check_pending) {
        // a deferred density check: its rejection takes precedence over a
        // pseudo-inverse that failed on the rejected coefficients
        c->check_pending = false;
        PP_TRY(coeff_verdict(c, true, c->check_rho_count));
    }
    if (prc != PP_OK)
        return prc;
    S.nb = std::sqrt(c->hscal[S_BB]);
    S.rel = (S.nb > 0.0) ? std::sqrt(c->hscal[S_RR]) / S.nb : 0.0;
    return PP_OK;
}

// The loop launches an iteration before knowing whether the previous one
// converged only while the last residual exceeds the tolerance by this
// factor times the square of the last measured reduction per iteration, so
// that the next iteration is needed unless convergence suddenly speeds up
// more than threefold (which then costs one extra iteration).
constexpr double SPECULATE = 10.0;

template <typename T>
int pcg_loop(pp_ctx *c, Hier &H, double *x, double tol, SolveState &S)
{
    using D = typename DirT<T>::type;
    hipStream_t s = c->stream;
    const double ih2 = 1.0 / (c->grid.h * c->grid.h);
    const int np = nparts(c);
    LevelBuf &v0 = H.lev[0];
    if (!c->scale_queued)
        launch_scale_T<T>(c->N, c->r64, (T *)v0.r, c->scal, s);
    c->scale_queued = false;
    bool first = true;
    D *dold = (D *)c->d64, *dnew = (D *)c->d64b;
    int since = 0;
    double window = S.rel;
    // Iterations are launched ahead of the host's convergence test while the
    // last known residual is far above the tolerance: the scalars of each
    // iteration are copied to a pinned slot of their own, and the host folds
    // them in one iteration late, so the GPU does not idle during the test.
    int launched = 0, seen = 0;
    double rate = 0.0;   // residual reduction of the last folded iteration (0: none yet)
    auto launch_iteration = [&]() -> int {
        // r . z comes from the V-cycle's last fine-level pass where that pass
        // can form it, else from its own kernel
        c->dot_on = true;
        c->dot_np = 0;
        const int vrc = vcycle_run<T>(c, H);
        c->dot_on = false;
        PP_TRY(vrc);
        if (S.st)
            S.st->vcycles++;
        int nrz = c->dot_np, op = OP_RZ_T;
        if (nrz == 0) {
            launch_dot_rz<T>(c->d, c->r64, (const T *)v0.cur, c->part, s);
            nrz = np;
            op = OP_RZ;
        }
        launch_finalize(c->part, c->pstride, nrz, op, 0, (double)c->N, first ? 1 : 0, c->scal, s);
        int npd;
        {
            KT t(c, PP_KT_OUTER_APPLY, true);
            // the iterate takes the pending directions two at a time: the
            // passes of odd iterations hold theirs, those of even ones apply
            // the last two
            const int mode = first ? DIR_FIRST : ((launched & 1) ? DIR_HOLD : DIR_TWO);
            if (!op_rho(c))
                PP_TRY(ensure_b64(c));
            npd = launch_dir_apply<T>(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2],
                                      op_rho(c), (const T *)v0.cur, dold, dnew, c->q64, x,
                                      c->sig_on ? c->sig[0] : nullptr, c->scal, mode, ih2, c->part,
                                      c->pstride, s);
        }
        first = false;
        launch_finalize(c->part, c->pstride, npd, OP_ALPHA, 0, (double)c->N, 0, c->scal, s);
        {
            KT t(c, PP_KT_OUTER_UPDATE, true);
            launch_pcg_update<T>(c->d, c->q64, c->r64, (T *)v0.r, c->scal, c->part, s);
        }
        std::swap(dold, dnew);
        // the finalising kernel also writes the iteration's scalars to their
        // pinned slot (no copy of its own on the stream)
        const int slot = launched & 1;
        c->iter_ticket[slot] = ++c->ticket;
        launch_finalize(c->part, c->pstride, np, OP_UPDATE, 0, (double)c->N, 0, c->scal, s,
                        c->hiter + slot * HSLOT, c->iter_ticket[slot]);
        PP_HIP(hipEventRecord(c->iter_ev[slot], s));
        ++launched;
        return check_launch("pcg iteration");
    };
    // fold the oldest unseen iteration into S: CONVERGED, PP_OK (go on),
    // STAGNATED or an error
    auto process = [&]() -> int {
        const int slot = seen & 1;
        PP_TRY(wait_ticket(c->hiter + slot * HSLOT + S_NSLOTS, c->iter_ticket[slot],
                           c->iter_ev[slot]));
        ++seen;
        S.it++;
        const double before = S.rel;
        S.rel = std::sqrt(c->hiter[slot * HSLOT + S_RR]) / S.nb;
        rate = (S.rel > 0.0) ? std::max(1.0, before / S.rel) : INFINITY;
        record(S);
        if (S.rel <= tol)
            return CONVERGED;
        return check_progress(S, 8, since, window);
    };
    int rc = PP_OK;
    for (;;) {
        if (S.it + (launched - seen) >= c->opts.max_outer) {
            rc = (seen < launched) ? process() : PP_OK;
            rc = (rc == CONVERGED) ? PP_OK
                                   : (rc == PP_OK ? fail(PP_ENOCONV,
                                                         "no convergence within max_outer iterations")
                                                  : rc);
            break;
        }
        rc = launch_iteration();
        if (rc != PP_OK)
            return rc;
        if (launched - seen == 2) {
            // the previous iteration: a convergence or stagnation stop it
            // calls for waits for the one now in flight, whose update the
            // iterate already carries; an error ends the loop at once
            rc = process();
            if (rc == CONVERGED || rc == STAGNATED)
                rc = process();
            if (rc != PP_OK)
                break;
        }
        if (launched - seen == 1) {
            if (rate > 0.0 && S.rel > SPECULATE * rate * rate * tol &&
                S.it + 1 < c->opts.max_outer)
                continue;   // the iteration after this one is needed either way
            rc = process();
            if (rc != PP_OK)
                break;
        }
    }
    if (rc == CONVERGED)
        rc = PP_OK;
    // the updates of the iterate still pending: the last direction (in dold
    // after the swap), and after an odd last iteration also the one before it
    // (in dnew), whose pass held it
    if (launched > 0) {
        const bool two = ((launched - 1) & 1) != 0;
        launch_axpy_dir<D>(c->N, dold, two ? dnew : nullptr, x, c->scal, s);
        PP_TRY(check_launch("pcg final update"));
    }
    return rc;
}

template <typename T>
int dc_loop(pp_ctx *c, Hier &H, const double *rhs, double *x, double tol, SolveState &S)
{
    hipStream_t s = c->stream;
    const double ih2 = 1.0 / (c->grid.h * c->grid.h);
    const int np = nparts(c);
    LevelBuf &v0 = H.lev[0];
    launch_scale_T<T>(c->N, c->r64, (T *)v0.r, c->scal, s);
    int since = 0;
    double window = S.rel;
    for (;;) {
        if (S.it >= c->opts.max_outer)
            return fail(PP_ENOCONV, "no convergence within max_outer iterations");
        PP_TRY(vcycle_run<T>(c, H));
        if (S.st)
            S.st->vcycles++;
        launch_axpy_T<T>(c->N, (const T *)v0.cur, x, c->scal, s);
        PP_TRY(ensure_b64(c));
        {
            KT t(c, PP_KT_OUTER_APPLY, true);
            launch_residual_T<T>(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2], rhs,
                                 c->scal, x, c->sig_on ? c->sig[0] : nullptr,
                                 c->gen ? c->act : nullptr, (T *)v0.r, ih2, c->part, s);
        }
        launch_finalize(c->part, c->pstride, np, OP_DC, 0, (double)c->N, 0, c->scal, s);
        PP_TRY(check_launch("defect-correction iteration"));
        PP_TRY(read_scal(c));
        S.it++;
        S.rel = std::sqrt(c->hscal[S_RR]) / S.nb;
        record(S);
        if (S.rel <= tol)
            return PP_OK;
        int rc = check_progress(S, 6, since, window);
        if (rc != PP_OK)
            return rc;
    }
}

int run_loop(pp_ctx *c, Hier &H, const double *rhs, double *x, double tol, SolveState &S)
{
    if (c->opts.outer == PP_OUTER_PCG) {
        switch (H.st) {
        case ST_F64: return pcg_loop<double>(c, H, x, tol, S);
        case ST_F32: return pcg_loop<float>(c, H, x, tol, S);
        default: return pcg_loop<_Float16>(c, H, x, tol, S);
        }
    }
    switch (H.st) {
    case ST_F64: return dc_loop<double>(c, H, rhs, x, tol, S);
    case ST_F32: return dc_loop<float>(c, H, rhs, x, tol, S);
    default: return dc_loop<_Float16>(c, H, rhs, x, tol, S);
    }
}

// Singular operator: remove the mean of x (over the active cells of the
// general operator).  General operator: excluded cells are set to 0.
// xsum_parts > 0: the partial sums of x are already in the third partials
// row (the residual kernel formed them), that many of them.
int gauge(pp_ctx *c, double *x, int xsum_parts)
{
    const unsigned char *act = c->gen ? c->act : nullptr;
    if (!c->gen || c->singular) {
        if (xsum_parts > 0) {
            launch_finalize(c->part + 2 * c->pstride, c->pstride, xsum_parts, OP_MEAN, S_XMEAN,
                            c->gen ? c->nact : (double)c->N, 0, c->scal, c->stream);
        } else {
            launch_sum(c->d, x, act, c->part, c->stream);
            launch_finalize(c->part, c->pstride, nparts(c), OP_MEAN, S_XMEAN,
                            c->gen ? c->nact : (double)c->N, 0, c->scal, c->stream);
        }
        launch_sub_mean(c->N, x, c->scal, S_XMEAN, act, c->stream);
    } else {
        launch_sub_mean(c->N, x, c->scal, -1, act, c->stream);
    }
    return check_launch("gauge");
}

// tail (may be null): work to queue behind the result; *tail_queued tells
// whether it was queued behind the final iterate (else the caller queues it)
// mean_ready: scal[S_MEAN] already holds the mean of rhs (pp_step's
// divergence formed it)
// the hierarchy a solve starts with, and the outer loop's first step on it:
// the residual divided by its RMS into level 0's right-hand side
Hier *first_hier(pp_ctx *c) { return (c->opts.precision == PP_FP64) ? &c->h64 : &c->hmix; }

void queue_scale_T(pp_ctx *c, Hier &H0, hipStream_t s)
{
    void *rT = H0.lev[0].r;
    switch (H0.st) {
    case ST_F64: launch_scale_T<double>(c->N, c->r64, (double *)rT, c->scal, s); break;
    case ST_F32: launch_scale_T<float>(c->N, c->r64, (float *)rT, c->scal, s); break;
    default: launch_scale_T<_Float16>(c->N, c->r64, (_Float16 *)rT, c->scal, s); break;
    }
}

int solve_impl(pp_ctx *c, const double *rhs, double *x, double tol, pp_stats *st, bool warm,
               const Tail *tail = nullptr, bool *tail_queued = nullptr, bool mean_ready = false)
{
    if (tail_queued)
        *tail_queued = false;
    const auto t0 = std::chrono::steady_clock::now();
    if (st) {
        std::memset(st, 0, sizeof(*st));
    }
    SolveState S{0.0, 0.0, INFINITY, 0, st};
    // the mean of the right-hand side is removed when the operator is
    // singular (over the active cells for the general operator)
    if (!mean_ready) {
        if (!c->gen || c->singular) {
            launch_sum(c->d, rhs, c->gen ? c->act : nullptr, c->part, c->stream);
            launch_finalize(c->part, c->pstride, nparts(c), OP_MEAN, S_MEAN,
                            c->gen ? c->nact : (double)c->N, 0, c->scal, c->stream);
        } else {
            launch_fill(c->scal + S_MEAN, 1, 0.0, c->stream);
        }
    }
    if (c->gen && warm)
        launch_mask(c->N, x, c->act, c->stream);   // excluded cells of a warm start are not read
    // The outer loop's first step, the residual scaled by its RMS into the
    // V-cycle's right-hand side, needs only values the device holds: it is
    // queued before the host waits for the initial residual, so the GPU has it
    // to work on meanwhile (if that residual is already small enough, nothing
    // reads it)
    Hier *H0 = first_hier(c);
    c->scale_queued = false;
    const Tail pre = [c, H0]() -> int {
        queue_scale_T(c, *H0, c->stream);
        c->scale_queued = true;
        return check_launch("scale");
    };
    const bool pcg = c->opts.outer == PP_OUTER_PCG && H0->present;
    PP_TRY(true_residual(c, rhs, x, !warm, S, false, nullptr, pcg ? &pre : nullptr));
    int rc = PP_OK;
    bool gauged = false;   // x is gauged and unchanged since
    if (!(S.nb > 0.0)) {
        // b = 0 after mean removal: the mean-zero solution is 0
        launch_fill(x, c->N, 0.0, c->stream);
        PP_TRY(check_launch("fill"));
        S.rel = 0.0;
    } else if (S.rel > tol) {
        Hier *H = (c->opts.precision == PP_FP64) ? &c->h64 : &c->hmix;
        S.best = S.rel;
        for (int restart = 0;; ++restart) {
            gauged = false;
            rc = run_loop(c, *H, rhs, x, tol, S);
            if (rc == PP_OK) {
                if (c->opts.outer == PP_OUTER_DC)
                    break;   // DC residuals are true residuals already
                // recurrences drift from the true residual: confirm it (the
                // gauge goes in the same queue)
                PP_TRY(true_residual(c, rhs, x, false, S, true, tail));
                gauged = true;
                if (S.rel <= tol)
                    break;
                if (restart >= 4) {
                    rc = fail(PP_ENOCONV, "true residual stays above tol after restarts");
                    break;
                }
                continue;
            }
            if (rc == STAGNATED) {
                if (H != &c->h64 && c->opts.fallback && c->h64.present) {
                    PP_TRY(ensure_b64(c));     // the FP64 hierarchy's fine level
                    H = &c->h64;
                    if (st)
                        st->fell_back = 1;
                    PP_TRY(true_residual(c, rhs, x, false, S));
                    if (S.rel <= tol) {
                        rc = PP_OK;
                        break;
                    }
                    continue;
                }
                rc = fail(PP_ENOCONV, "outer iteration stagnated");
            }
            break;
        }
    }
    if ((rc == PP_OK || rc == PP_ENOCONV) && !gauged)
        PP_TRY(gauge(c, x));
    if (tail_queued)
        *tail_queued = gauged && tail;   // queued at the last confirmation, x unchanged since
    // the result is known; the gauge may still be queued (stream order).
    // Timer events are read when queried, or when their pool runs out.
    if (st) {
        st->outer_iters = S.it;
        st->rel_res = S.rel;
        st->status = rc;
        st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

int check_ctx(const pp_ctx *c)
{
    if (!c)
        return fail(PP_EINVAL, "context is NULL");
    return PP_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void pp_opts_default(pp_opts *o)
{
    if (!o)
        return;
    std::memset(o, 0, sizeof(*o));
    o->precision = PP_MIXED_FP32;
    o->outer = PP_OUTER_PCG;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->max_outer = 500;
    o->warm_start = 0;
    o->fallback = 1;
    o->coarse_graph = 0;   // eager launches: the graph's exit costs more than its launches save
    o->nu_coarse = 4;
    // measured at 256^3 (layer and droplets): 1.1-1.4 all take 7 outer
    // iterations where plain Gauss-Seidel (1.0) takes 8; 1.2 sits mid-plateau
    o->omega = 1.2;
    o->cycle = PP_CYCLE_V;
    o->coarsest = 64;
}

const char *pp_strerror(int status)
{
    switch (status) {
    case PP_OK: return "ok";
    case PP_EINVAL: return "invalid argument";
    case PP_ENOMEM: return "out of memory";
    case PP_EHIP: return "HIP runtime error";
    case PP_ENOCONV: return "not converged";
    case PP_EDIVERGED: return "diverged";
    default: return "unknown status";
    }
}

const char *pp_last_error(void) { return g_err.c_str(); }

int pp_face_coeffs(const pp_grid *grid, const double *rho, double *bx, double *by, double *bz,
                   void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!rho || !bx || !by || !bz)
        return fail(PP_EINVAL, "pp_face_coeffs: NULL array");
    launch_face_coeffs(to_dims(grid), to_bc(grid), rho, bx, by, bz, (hipStream_t)hip_stream);
    return check_launch("pp_face_coeffs");
}

void pp_destroy(pp_ctx *c)
{
    if (!c)
        return;
    (void)hipStreamSynchronize(c->stream);
    for (Hier *H : {&c->hmix, &c->h64})
        if (H->coarse_exec)
            (void)hipGraphExecDestroy(H->coarse_exec);
    for (auto &e : c->ev) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (void *p : c->allocs)
        (void)hipFree(p);
    if (c->hscal)
        (void)hipHostFree(c->hscal);
    if (c->hcoarse)
        (void)hipHostFree(c->hcoarse);
    if (c->hpinv)
        (void)hipHostFree(c->hpinv);
    if (c->hiter)
        (void)hipHostFree(c->hiter);
    for (hipEvent_t e : c->iter_ev)
        if (e)
            (void)hipEventDestroy(e);
    if (c->scal_ev)
        (void)hipEventDestroy(c->scal_ev);
    if (c->coarse_ev)
        (void)hipEventDestroy(c->coarse_ev);
    if (c->pinv_ev)
        (void)hipEventDestroy(c->pinv_ev);
    if (c->copy_stream)
        (void)hipStreamDestroy(c->copy_stream);
    if (c->aux_start)
        (void)hipEventDestroy(c->aux_start);
    if (c->aux_done)
        (void)hipEventDestroy(c->aux_done);
    if (c->aux_stream)
        (void)hipStreamDestroy(c->aux_stream);
    if (c->pinv_free)
        (void)hipEventDestroy(c->pinv_free);
    delete c;
}

}  // extern "C"

namespace {

int setup_impl(const pp_grid *grid, const double *bx, const double *by, const double *bz,
               const double *sg, bool gen, const pp_opts *opts, void *hip_stream, pp_ctx **out)
{
    if (!out)
        return fail(PP_EINVAL, "pp_setup: out is NULL");
    *out = nullptr;
    int nlev = 0;
    Dims ld[MAXLEV];
    double lh[MAXLEV];
    pp_opts o;
    if (opts)
        o = *opts;
    else
        pp_opts_default(&o);
    PP_TRY(validate_opts(&o));
    PP_TRY(validate_grid(grid, &nlev, ld, lh, o.coarsest));
    if (!bx || !by || !bz)
        return fail(PP_EINVAL, "pp_setup: NULL beta array");

    pp_ctx *c = new pp_ctx();
    c->grid = *grid;
    c->opts = o;
    c->stream = (hipStream_t)hip_stream;
    c->d = to_dims(grid);
    c->bc = to_bc(grid);
    c->N = cells(c->d);
    c->nlev = nlev;
    for (int l = 0; l < nlev; ++l) {
        c->ld[l] = ld[l];
        c->lh[l] = lh[l];
    }
    c->ncoarse = (int)cells(ld[nlev - 1]);
    c->timing = false;
    c->ev_used = 0;
    c->gen = gen;
    c->sig_on = gen && sg != nullptr;
    c->singular = true;
    c->act = nullptr;
    c->nact = (double)c->N;
    for (int l = 0; l < MAXLEV; ++l)
        c->sig[l] = nullptr;
    int rc = PP_OK;
    auto bail = [&](int code) {
        pp_destroy(c);
        return code;
    };
    for (int l = 0; l < nlev && rc == PP_OK; ++l)
        for (int m = 0; m < 3 && rc == PP_OK; ++m)
            rc = dev_alloc_t(c, &c->chain[l][m], sizeof(double) * cells(ld[l]));
    for (int l = 0; l < MAXLEV; ++l)
        c->pw[l] = nullptr;
    for (int l = 0; l + 1 < nlev && rc == PP_OK; ++l)
        rc = dev_alloc_t(c, &c->pw[l], sizeof(unsigned) * cells(ld[l]));
    for (int l = 0; l < nlev && rc == PP_OK && c->sig_on; ++l)
        rc = dev_alloc_t(c, &c->sig[l], sizeof(double) * cells(ld[l]));
    if (rc == PP_OK && gen)
        rc = dev_alloc_t(c, &c->act, c->N);
    if (rc == PP_OK && (o.precision == PP_FP64 || o.fallback))
        rc = alloc_hier(c, c->h64, ST_F64);
    if (rc == PP_OK && o.precision != PP_FP64)
        rc = alloc_hier(c, c->hmix, o.precision == PP_MIXED_FP32 ? ST_F32 : ST_F16);
    if (rc == PP_OK)
        rc = dev_alloc_t(c, &c->pinv, sizeof(double) * (size_t)c->ncoarse * c->ncoarse);
    if (rc == PP_OK)
        rc = dev_alloc_t(c, &c->r64, sizeof(double) * c->N);
    if (rc == PP_OK)
        rc = dev_alloc_t(c, &c->d64, sizeof(double) * c->N);
    if (rc == PP_OK)
        rc = dev_alloc_t(c, &c->d64b, sizeof(double) * c->N);
    if (rc == PP_OK)
        rc = dev_alloc_t(c, &c->q64, sizeof(double) * c->N);
    c->pstride = grid_blocks(red_grid(c->d));
    if (rc == PP_OK)
        rc = dev_alloc_t(c, &c->part, sizeof(double) * 6 * c->pstride);   // rows 3..5: pp_step's side stream
    if (rc == PP_OK)
        rc = dev_alloc_t(c, &c->scal, sizeof(double) * S_NSLOTS);
    if (rc != PP_OK)
        return bail(rc);
    if (hipHostMalloc((void **)&c->hscal, sizeof(double) * HSLOT, hipHostMallocCoherent) !=
        hipSuccess) {
        c->hscal = nullptr;
        return bail(fail(PP_ENOMEM, "hipHostMalloc failed"));
    }
    if (hipHostMalloc((void **)&c->hcoarse, sizeof(double) * 4 * (size_t)c->ncoarse,
                      hipHostMallocCoherent) != hipSuccess) {
        c->hcoarse = nullptr;
        return bail(fail(PP_ENOMEM, "hipHostMalloc failed"));
    }
    if (hipHostMalloc((void **)&c->hpinv, sizeof(double) * (size_t)c->ncoarse * c->ncoarse,
                      hipHostMallocDefault) != hipSuccess) {
        c->hpinv = nullptr;
        return bail(fail(PP_ENOMEM, "hipHostMalloc failed"));
    }
    // coherent: the finalising kernel writes the iteration scalars here itself
    if (hipHostMalloc((void **)&c->hiter, sizeof(double) * 2 * HSLOT, hipHostMallocCoherent) !=
        hipSuccess) {
        c->hiter = nullptr;
        return bail(fail(PP_ENOMEM, "hipHostMalloc failed"));
    }
    // tickets start at 1 and only grow: no flag holds one before its kernel runs
    std::fill(c->hscal, c->hscal + HSLOT, 0.0);
    std::fill(c->hiter, c->hiter + 2 * HSLOT, 0.0);
    c->ticket = 0.0;
    for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&c->iter_ev[i], hipEventDisableTiming) != hipSuccess) {
            c->iter_ev[i] = nullptr;
            return bail(fail(PP_EHIP, "hipEventCreateWithFlags failed"));
        }
    if (hipEventCreateWithFlags(&c->scal_ev, hipEventDisableTiming) != hipSuccess) {
        c->scal_ev = nullptr;
        return bail(fail(PP_EHIP, "hipEventCreateWithFlags failed"));
    }
    if (hipEventCreateWithFlags(&c->coarse_ev, hipEventDisableTiming) != hipSuccess) {
        c->coarse_ev = nullptr;
        return bail(fail(PP_EHIP, "hipEventCreateWithFlags failed"));
    }
    if (hipEventCreateWithFlags(&c->pinv_ev, hipEventDisableTiming) != hipSuccess) {
        c->pinv_ev = nullptr;
        return bail(fail(PP_EHIP, "hipEventCreateWithFlags failed"));
    }
    // default priority, like every stream here
    if (hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        c->copy_stream = nullptr;
        return bail(fail(PP_EHIP, "hipStreamCreateWithFlags failed"));
    }
    if (hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking) != hipSuccess) {
        c->aux_stream = nullptr;
        return bail(fail(PP_EHIP, "hipStreamCreateWithFlags failed"));
    }
    for (hipEvent_t *ev : {&c->aux_start, &c->aux_done, &c->pinv_free}) {
        if (hipEventCreateWithFlags(ev, hipEventDisableTiming) != hipSuccess) {
            *ev = nullptr;
            return bail(fail(PP_EHIP, "hipEventCreateWithFlags failed"));
        }
    }
    if (hipMemsetAsync(c->scal, 0, sizeof(double) * S_NSLOTS, c->stream) != hipSuccess)
        return bail(fail(PP_EHIP, "hipMemsetAsync failed"));
    rc = gen ? load_coeffs_general(c, bx, by, bz, sg) : load_coeffs(c, bx, by, bz);
    if (rc == PP_OK)
        rc = capture_graphs(c);
    if (rc != PP_OK)
        return bail(rc);
    *out = c;
    return PP_OK;
}

// Arguments of the two-sweep pass that forms r . e_out (both entry points):
// every check of pp_k_smooth2_fused_f32 plus the output pointer.  On success
// *nparts_max bounds the number of workgroup partial sums the launch writes.
int check_smooth2_dot(const char *who, const pp_grid *grid, const float *bx, const float *by,
                      const float *bz, const float *r, const float *e_in, const float *e_out,
                      int32_t first_colour, double omega, const double *dot, size_t *nparts_max)
{
    const std::string w(who);
    if (!omega_ok(omega))
        return fail(PP_EINVAL, w + ": omega must be in (0, 2)");
    if (!dot)
        return fail(PP_EINVAL, w + ": NULL array");
    if ((uintptr_t)dot & 7)
        return fail(PP_EINVAL, w + ": dot must be 8-byte aligned");
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!fused_plane_fits(to_dims(grid), sizeof(float)))
        return fail(PP_EINVAL, w + ": an x-y plane must stay below 2^31 bytes");
    if (!bx || !by || !bz || !r || !e_in || !e_out)
        return fail(PP_EINVAL, w + ": NULL array");
    if (((uintptr_t)bx | (uintptr_t)by | (uintptr_t)bz | (uintptr_t)r | (uintptr_t)e_in |
         (uintptr_t)e_out) & 15)
        return fail(PP_EINVAL, w + ": arrays must be 16-byte aligned");
    if (e_in == e_out)
        return fail(PP_EINVAL, w + ": e_in and e_out must not alias");
    if (first_colour != 0 && first_colour != 1)
        return fail(PP_EINVAL, w + ": first_colour must be 0 or 1");
    if (grid->n[0] % 2)
        return fail(PP_EINVAL, w + ": nx must be even");
    for (int m = 0; m < 3; ++m)
        if (grid->bc[m] == PP_PERIODIC && grid->n[m] % 2)
            return fail(PP_EINVAL, w + ": periodic directions need an even cell count");
    const Dims d = to_dims(grid);
    if (!fused2_fits(d))
        return fail(PP_EINVAL, w + ": every cell count must be >= 8");
    // at most one partial per workgroup: tiles x z chunks of >= 8 planes
    *nparts_max = (size_t)((d.nx + 63) / 64) * ((d.ny + 7) / 8) * ((d.nz + 7) / 8);
    return PP_OK;
}

// Workgroup partial sums of pp_k_smooth2_fused_dot_f32_noalloc live in this
// fixed device array (512 KiB; each GPU the library runs on holds its own
// copy until the process ends) instead of a buffer allocated per call.  Host
// code must not pass `scratch` itself to a kernel: its device address comes
// from hipGetSymbolAddress, taken once per device.
constexpr size_t NOALLOC_PARTS = 65536;
static __device__ __align__(256) double scratch[NOALLOC_PARTS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[MAX_DEVICES] = {};

// Device address of `scratch` on the device that owns stream s (which must be
// the calling thread's current device), looked up on the first call there.
int noalloc_scratch(hipStream_t s, double **out)
{
    int dev = 0;
    PP_HIP(hipGetDevice(&dev));
    if (s) {
        int sdev = -1;
        PP_HIP(hipStreamGetDevice(s, &sdev));
        if (sdev != dev)
            return fail(PP_EINVAL, "pp_k_smooth2_fused_dot_f32_noalloc: the stream belongs to "
                                   "device " + std::to_string(sdev) + ", the current device is " +
                                   std::to_string(dev));
    }
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(PP_EINVAL, "pp_k_smooth2_fused_dot_f32_noalloc: device index beyond " +
                                   std::to_string(MAX_DEVICES - 1));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        PP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return fail(PP_EHIP, "pp_k_smooth2_fused_dot_f32_noalloc: no device address for the "
                                 "scratch array");
        g_scratch_addr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_addr[dev];
    return PP_OK;
}

}  // namespace

extern "C" {

int pp_setup(const pp_grid *grid, const double *bx, const double *by, const double *bz,
             const pp_opts *opts, void *hip_stream, pp_ctx **out)
{
    return setup_impl(grid, bx, by, bz, nullptr, false, opts, hip_stream, out);
}

int pp_setup_general(const pp_grid *grid, const double *bx, const double *by, const double *bz,
                     const double *sigma, const pp_opts *opts, void *hip_stream, pp_ctx **out)
{
    return setup_impl(grid, bx, by, bz, sigma, true, opts, hip_stream, out);
}

int pp_update_coeffs(pp_ctx *c, const double *bx, const double *by, const double *bz)
{
    PP_TRY(check_ctx(c));
    if (!bx || !by || !bz)
        return fail(PP_EINVAL, "pp_update_coeffs: NULL beta array");
    if (c->gen) {
        if (c->sig_on)
            return fail(PP_EINVAL, "pp_update_coeffs: the context has a diagonal term; use "
                                   "pp_update_general");
        return load_coeffs_general(c, bx, by, bz, nullptr);
    }
    return load_coeffs(c, bx, by, bz);
}

int pp_update_density(pp_ctx *c, const double *rho)
{
    PP_TRY(check_ctx(c));
    if (!rho)
        return fail(PP_EINVAL, "pp_update_density: NULL rho");
    if (c->gen)
        return fail(PP_EINVAL, "pp_update_density: a general context takes its coefficients "
                               "from pp_update_general");
    const double *src[3] = {nullptr, nullptr, nullptr};
    return load_coeffs_impl(c, src, rho);
}

int pp_update_general(pp_ctx *c, const double *bx, const double *by, const double *bz,
                      const double *sigma)
{
    PP_TRY(check_ctx(c));
    if (!c->gen)
        return fail(PP_EINVAL, "pp_update_general: the context was made by pp_setup");
    if (!bx || !by || !bz)
        return fail(PP_EINVAL, "pp_update_general: NULL beta array");
    if ((sigma != nullptr) != c->sig_on)
        return fail(PP_EINVAL, c->sig_on ? "pp_update_general: the context has a diagonal term: "
                                           "sigma must be given"
                                         : "pp_update_general: the context has no diagonal term: "
                                           "sigma must be NULL");
    return load_coeffs_general(c, bx, by, bz, sigma);
}

int pp_divergence(pp_ctx *c, const double *ux, const double *uy, const double *uz, double scale,
                  double *out)
{
    PP_TRY(check_ctx(c));
    if (!ux || !uy || !uz || !out)
        return fail(PP_EINVAL, "pp_divergence: NULL array");
    if (!std::isfinite(scale))
        return fail(PP_EINVAL, "pp_divergence: scale must be finite");
    const double *const *bt = c->chain[0];
    launch_divergence(c->d, c->bc, ux, uy, uz, scale / c->grid.h, c->gen ? bt[0] : nullptr,
                      c->gen ? bt[1] : nullptr, c->gen ? bt[2] : nullptr, out, c->stream);
    return check_launch("pp_divergence");
}

int pp_apply(pp_ctx *c, const double *x, double *y)
{
    PP_TRY(check_ctx(c));
    if (!x || !y)
        return fail(PP_EINVAL, "pp_apply: NULL array");
    if (x == y)
        return fail(PP_EINVAL, "pp_apply: x and out must not alias");
    PP_TRY(ensure_b64(c));
    launch_apply(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2], x,
                 c->sig_on ? c->sig[0] : nullptr, y, 1.0 / (c->grid.h * c->grid.h), c->stream);
    return check_launch("pp_apply");
}

int pp_solve(pp_ctx *c, const double *rhs, double *p, double tol, pp_stats *st)
{
    PP_TRY(check_ctx(c));
    if (!rhs || !p)
        return fail(PP_EINVAL, "pp_solve: NULL array");
    if (rhs == p)
        return fail(PP_EINVAL, "pp_solve: rhs and p must not alias");
    if (!(tol > 0.0 && tol < 1.0))
        return fail(PP_EINVAL, "pp_solve: tol must be in (0, 1)");
    return solve_impl(c, rhs, p, tol, st, c->opts.warm_start != 0);
}

int pp_project(pp_ctx *c, const double *usx, const double *usy, const double *usz, const double *p,
               double dt, double *ux, double *uy, double *uz)
{
    PP_TRY(check_ctx(c));
    if (!usx || !usy || !usz || !p || !ux || !uy || !uz)
        return fail(PP_EINVAL, "pp_project: NULL array");
    if (p == ux || p == uy || p == uz)
        return fail(PP_EINVAL, "pp_project: p must not alias the output");
    if (!std::isfinite(dt))
        return fail(PP_EINVAL, "pp_project: dt must be finite");
    if (!op_rho(c))
        PP_TRY(ensure_b64(c));
    launch_project(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2], op_rho(c), usx, usy,
                   usz, p, dt / c->grid.h, ux, uy, uz, c->stream);
    return check_launch("pp_project");
}

int pp_step(pp_ctx *c, const double *rho, const double *usx, const double *usy,
            const double *usz, double dt, double tol, double *rhs, double *p, double *ux,
            double *uy, double *uz, pp_stats *st)
{
    PP_TRY(check_ctx(c));
    if (!rho || !usx || !usy || !usz || !rhs || !p || !ux || !uy || !uz)
        return fail(PP_EINVAL, "pp_step: NULL array");
    if (c->gen)
        return fail(PP_EINVAL, "pp_step: a general context takes its coefficients from "
                               "pp_update_general");
    if (!(std::isfinite(dt) && dt != 0.0 && std::isfinite(1.0 / dt)))
        return fail(PP_EINVAL, "pp_step: dt must be finite and nonzero");
    if (!(tol > 0.0 && tol < 1.0))
        return fail(PP_EINVAL, "pp_step: tol must be in (0, 1)");
    const double *outs[5] = {rhs, p, ux, uy, uz};
    const double *ins[4] = {rho, usx, usy, usz};
    for (int a = 0; a < 5; ++a) {
        for (int b = a + 1; b < 5; ++b)
            if (outs[a] == outs[b])
                return fail(PP_EINVAL, "pp_step: rhs, p and the u arrays must be distinct");
        for (int b = 0; b < 4; ++b)
            if (outs[a] == ins[b] && !(a >= 2 && b == a - 1))
                return fail(PP_EINVAL, "pp_step: an output aliases an input (only u_m may "
                                       "alias us_m)");
    }
    // The divergence needs only u*: it runs on a side stream beside the
    // coefficient load (both stream memory below the HBM rate, and the load's
    // coarse levels are short latency-bound launches), with its partial sums
    // in rows 3..5 of the reduction buffer, which the load does not use, and
    // its mean in a scalar slot the load does not write.  It also sums what it writes, as the solve's pass over the
    // right-hand side would (same blocks, same order, same bits).
    // A cold start's initial residual, b - mean b with p = 0, needs no
    // coefficients either: it follows on the side stream, with (for PCG) the
    // outer loop's first step, and the solve takes them from there.
    PP_HIP(hipEventRecord(c->aux_start, c->stream));
    PP_HIP(hipStreamWaitEvent(c->aux_stream, c->aux_start, 0));
    double *apart = c->part + 3 * c->pstride;
    const int np = launch_divergence_sum(c->d, c->bc, usx, usy, usz, (1.0 / dt) / c->grid.h, rhs,
                                         apart, c->aux_stream);
    launch_finalize(apart, c->pstride, np, OP_MEAN, S_MEAN, (double)c->N, 0, c->scal,
                    c->aux_stream);
    c->init_queued = c->init_scaled = false;
    if (c->opts.warm_start == 0) {
        Hier *H0 = first_hier(c);
        const int npr = launch_residual(c->d, c->bc, nullptr, nullptr, nullptr, nullptr, rhs,
                                        c->scal, p, true, nullptr, nullptr, c->r64,
                                        1.0 / (c->grid.h * c->grid.h), apart, c->pstride,
                                        c->aux_stream);
        launch_finalize(apart, c->pstride, npr, OP_INIT, 0, (double)c->N, 0, c->scal,
                        c->aux_stream);
        c->init_queued = true;
        if (c->opts.outer == PP_OUTER_PCG && H0->present) {
            queue_scale_T(c, *H0, c->aux_stream);
            c->init_scaled = true;
        }
    }
    PP_HIP(hipEventRecord(c->aux_done, c->aux_stream));
    PP_TRY(check_launch("pp_step divergence"));
    // the coefficient load leaves its validity counts to the solve's first
    // wait, so the step waits on the host for the solve's results only
    const double *src[3] = {nullptr, nullptr, nullptr};
    const int lrc = load_coeffs_impl(c, src, rho, true);
    // the solve (and any later work on the stream) follows the side stream
    PP_HIP(hipStreamWaitEvent(c->stream, c->aux_done, 0));
    if (lrc != PP_OK)
        c->init_queued = c->init_scaled = false;
    PP_TRY(lrc);
    const Tail project = [&]() {
        if (!op_rho(c))
            PP_TRY(ensure_b64(c));
        launch_project(c->d, c->bc, c->chain[0][0], c->chain[0][1], c->chain[0][2], op_rho(c), usx,
                       usy, usz, p, dt / c->grid.h, ux, uy, uz, c->stream);
        return check_launch("pp_step projection");
    };
    // the projection is queued behind the confirmation of convergence, before
    // the host waits for it; a projection in place (u over u*) waits instead,
    // as it cannot be redone if the iterate goes on
    const bool in_place = ux == usx || uy == usy || uz == usz;
    bool queued = false;
    const int rc = solve_impl(c, rhs, p, tol, st, c->opts.warm_start != 0,
                              in_place ? nullptr : &project, &queued, true);
    if (rc != PP_OK && rc != PP_ENOCONV)
        return rc;
    if (!queued)
        PP_TRY(project());
    return rc;
}

int pp_solve_adjoint(pp_ctx *c, const double *p, const double *gp, double tol, double *grhs,
                     double *gbx, double *gby, double *gbz, pp_stats *st)
{
    PP_TRY(check_ctx(c));
    if (!p || !gp || !grhs || !gbx || !gby || !gbz)
        return fail(PP_EINVAL, "pp_solve_adjoint: NULL array");
    if (grhs == gp || grhs == p)
        return fail(PP_EINVAL, "pp_solve_adjoint: g_rhs must not alias p or g_p");
    if (!(tol > 0.0 && tol < 1.0))
        return fail(PP_EINVAL, "pp_solve_adjoint: tol must be in (0, 1)");
    int rc = solve_impl(c, gp, grhs, tol, st, false);
    if (rc != PP_OK && rc != PP_ENOCONV)
        return rc;
    const double *const *bt = c->chain[0];
    launch_adjoint_faces(c->d, c->bc, grhs, p, 1.0 / (c->grid.h * c->grid.h),
                         c->gen ? bt[0] : nullptr, c->gen ? bt[1] : nullptr,
                         c->gen ? bt[2] : nullptr, gbx, gby, gbz, c->stream);
    PP_TRY(check_launch("adjoint faces"));
    return rc;
}

int pp_levels(const pp_ctx *c, int32_t *nlevels)
{
    PP_TRY(check_ctx(c));
    if (!nlevels)
        return fail(PP_EINVAL, "pp_levels: NULL output");
    *nlevels = c->nlev;
    return PP_OK;
}

int pp_level_dims(const pp_ctx *c, int32_t level, int32_t dims[3])
{
    PP_TRY(check_ctx(c));
    if (!dims || level < 0 || level >= c->nlev)
        return fail(PP_EINVAL, "pp_level_dims: bad level or NULL output");
    dims[0] = c->ld[level].nx;
    dims[1] = c->ld[level].ny;
    dims[2] = c->ld[level].nz;
    return PP_OK;
}

int pp_memory(const pp_ctx *c, int64_t *bytes)
{
    PP_TRY(check_ctx(c));
    if (!bytes)
        return fail(PP_EINVAL, "pp_memory: NULL output");
    *bytes = c->bytes;
    return PP_OK;
}

// ---------------------------------------------------------------------------
// single-kernel entry points (pp_kernels.h)
// ---------------------------------------------------------------------------

int pp_k_smooth(const pp_grid *grid, const double *bx, const double *by, const double *bz,
                const double *r, double *e, int32_t sweeps, int32_t zero_init, double omega,
                void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!bx || !by || !bz || !r || !e)
        return fail(PP_EINVAL, "pp_k_smooth: NULL array");
    if (sweeps < 1)
        return fail(PP_EINVAL, "pp_k_smooth: sweeps must be >= 1");
    if (!omega_ok(omega))
        return fail(PP_EINVAL, "pp_k_smooth: omega must be in (0, 2)");
    for (int m = 0; m < 3; ++m)
        if (grid->bc[m] == PP_PERIODIC && grid->n[m] % 2)
            return fail(PP_EINVAL, "pp_k_smooth: periodic directions need an even cell count");
    const Dims d = to_dims(grid);
    const Bc bc = to_bc(grid);
    const double h2 = grid->h * grid->h;
    hipStream_t s = (hipStream_t)hip_stream;
    for (int sw = 0; sw < sweeps; ++sw) {
        const bool z = zero_init && sw == 0;
        launch_rbgs<double>(d, bc, bx, by, bz, r, e, nullptr, h2, omega, 0, z, false, s);
        launch_rbgs<double>(d, bc, bx, by, bz, r, e, nullptr, h2, omega, 1, false, z, s);
    }
    return check_launch("pp_k_smooth");
}

int pp_k_smooth_fused(const pp_grid *grid, const double *bx, const double *by, const double *bz,
                      const double *r, const double *e_in, double *e_out, int32_t first_colour,
                      int32_t zero_init, double omega, void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!bx || !by || !bz || !r || !e_in || !e_out)
        return fail(PP_EINVAL, "pp_k_smooth_fused: NULL array");
    if (!omega_ok(omega))
        return fail(PP_EINVAL, "pp_k_smooth_fused: omega must be in (0, 2)");
    if (((uintptr_t)bx | (uintptr_t)by | (uintptr_t)bz | (uintptr_t)r | (uintptr_t)e_in |
         (uintptr_t)e_out) & 15)
        return fail(PP_EINVAL, "pp_k_smooth_fused: arrays must be 16-byte aligned");
    if (e_in == e_out)
        return fail(PP_EINVAL, "pp_k_smooth_fused: e_in and e_out must not alias");
    if (first_colour != 0 && first_colour != 1)
        return fail(PP_EINVAL, "pp_k_smooth_fused: first_colour must be 0 or 1");
    if (grid->n[0] % 2)
        return fail(PP_EINVAL, "pp_k_smooth_fused: nx must be even (threads own x-pairs)");
    for (int m = 0; m < 3; ++m)
        if (grid->bc[m] == PP_PERIODIC && grid->n[m] % 2)
            return fail(PP_EINVAL, "pp_k_smooth_fused: periodic directions need an even cell count");
    if (!fused_plane_fits(to_dims(grid), sizeof(double)))
        return fail(PP_EINVAL, "pp_k_smooth_fused: an x-y plane must stay below 2^31 bytes");
    launch_rbgs_fused<double>(to_dims(grid), to_bc(grid), bx, by, bz, r, e_in, e_out, nullptr,
                              grid->h * grid->h, omega, first_colour, zero_init != 0,
                              (hipStream_t)hip_stream);
    return check_launch("pp_k_smooth_fused");
}

int pp_k_smooth2_fused_f32(const pp_grid *grid, const float *bx, const float *by, const float *bz,
                           const float *r, const float *e_in, float *e_out, int32_t first_colour,
                           int32_t zero_init, double omega, void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!bx || !by || !bz || !r || !e_in || !e_out)
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: NULL array");
    if (!omega_ok(omega))
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: omega must be in (0, 2)");
    if (((uintptr_t)bx | (uintptr_t)by | (uintptr_t)bz | (uintptr_t)r | (uintptr_t)e_in |
         (uintptr_t)e_out) & 15)
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: arrays must be 16-byte aligned");
    if (e_in == e_out)
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: e_in and e_out must not alias");
    if (first_colour != 0 && first_colour != 1)
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: first_colour must be 0 or 1");
    if (grid->n[0] % 2)
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: nx must be even (threads own x-pairs)");
    for (int m = 0; m < 3; ++m)
        if (grid->bc[m] == PP_PERIODIC && grid->n[m] % 2)
            return fail(PP_EINVAL,
                        "pp_k_smooth2_fused_f32: periodic directions need an even cell count");
    if (!fused2_fits(to_dims(grid)))
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: every cell count must be >= 8");
    if (!fused_plane_fits(to_dims(grid), sizeof(float)))
        return fail(PP_EINVAL, "pp_k_smooth2_fused_f32: an x-y plane must stay below 2^31 bytes");
    launch_rbgs_fused2<float>(to_dims(grid), to_bc(grid), bx, by, bz, r, e_in, e_out, nullptr,
                              grid->h * grid->h, omega, first_colour, zero_init != 0,
                              (hipStream_t)hip_stream);
    return check_launch("pp_k_smooth2_fused_f32");
}

int pp_k_smooth2_fused_dot_f32(const pp_grid *grid, const float *bx, const float *by,
                               const float *bz, const float *r, const float *e_in, float *e_out,
                               int32_t first_colour, double omega, double *dot, void *hip_stream)
{
    size_t nparts_max = 0;
    PP_TRY(check_smooth2_dot("pp_k_smooth2_fused_dot_f32", grid, bx, by, bz, r, e_in, e_out,
                             first_colour, omega, dot, &nparts_max));
    const Dims d = to_dims(grid);
    double *part = nullptr;
    PP_HIP(hipMalloc((void **)&part, sizeof(double) * nparts_max));
    hipStream_t s = (hipStream_t)hip_stream;
    const int np = launch_rbgs_fused2<float>(d, to_bc(grid), bx, by, bz, r, e_in, e_out, nullptr,
                                             grid->h * grid->h, omega, first_colour, false, s,
                                             part);
    int rc = PP_OK;
    if (np <= 0 || (size_t)np > nparts_max)
        rc = fail(PP_EHIP, "pp_k_smooth2_fused_dot_f32: unexpected workgroup count");
    else
        launch_finalize(part, (size_t)np, np, OP_STORE, 0, 1.0, 0, dot, s);
    const int rl = check_launch("pp_k_smooth2_fused_dot_f32");
    (void)hipStreamSynchronize(s);
    (void)hipFree(part);
    return rc != PP_OK ? rc : rl;
}

int pp_k_smooth2_fused_dot_f32_noalloc(const pp_grid *grid, const float *bx, const float *by,
                                       const float *bz, const float *r, const float *e_in,
                                       float *e_out, int32_t first_colour, double omega,
                                       double *dot, void *hip_stream)
{
    size_t nparts_max = 0;
    PP_TRY(check_smooth2_dot("pp_k_smooth2_fused_dot_f32_noalloc", grid, bx, by, bz, r, e_in,
                             e_out, first_colour, omega, dot, &nparts_max));
    if (nparts_max > NOALLOC_PARTS)
        return fail(PP_EINVAL, "pp_k_smooth2_fused_dot_f32_noalloc: the grid needs up to " +
                                   std::to_string(nparts_max) +
                                   " workgroup partial sums (ceil(nx/64) ceil(ny/8) ceil(nz/8)); "
                                   "the static scratch holds " +
                                   std::to_string(NOALLOC_PARTS));
    hipStream_t s = (hipStream_t)hip_stream;
    double *part = nullptr;
    PP_TRY(noalloc_scratch(s, &part));
    // the launch takes z chunks of at least 8 planes, so it never uses more
    // than nparts_max partial sums (checked above against the array size)
    const int np = launch_rbgs_fused2<float>(to_dims(grid), to_bc(grid), bx, by, bz, r, e_in,
                                             e_out, nullptr, grid->h * grid->h, omega,
                                             first_colour, false, s, part);
    PP_TRY(check_launch("pp_k_smooth2_fused_dot_f32_noalloc"));
    if (np <= 0 || (size_t)np > nparts_max)
        return fail(PP_EHIP, "pp_k_smooth2_fused_dot_f32_noalloc: unexpected workgroup count");
    // every partial the finalising sum reads was written by this launch
    launch_finalize(part, (size_t)np, np, OP_STORE, 0, 1.0, 0, dot, s);
    return check_launch("pp_k_smooth2_fused_dot_f32_noalloc");
}

int pp_k_resid_restrict(const pp_grid *grid, const double *bx, const double *by, const double *bz,
                        const double *e, const double *r, double *rH, void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!bx || !by || !bz || !e || !r || !rH)
        return fail(PP_EINVAL, "pp_k_resid_restrict: NULL array");
    if (((uintptr_t)bx | (uintptr_t)by | (uintptr_t)bz | (uintptr_t)e | (uintptr_t)r) & 15)
        return fail(PP_EINVAL, "pp_k_resid_restrict: arrays must be 16-byte aligned");
    for (int m = 0; m < 3; ++m)
        if (grid->n[m] % 2)
            return fail(PP_EINVAL, "pp_k_resid_restrict: the fine grid needs even cell counts");
    launch_resid_restrict<double>(to_dims(grid), to_bc(grid), bx, by, bz, e, r, nullptr, rH,
                                  1.0 / (grid->h * grid->h), (hipStream_t)hip_stream);
    return check_launch("pp_k_resid_restrict");
}

int pp_k_prolong_add(const pp_grid *grid, const double *eH, double *e, void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!eH || !e)
        return fail(PP_EINVAL, "pp_k_prolong_add: NULL array");
    for (int m = 0; m < 3; ++m)
        if (grid->n[m] % 2)
            return fail(PP_EINVAL, "pp_k_prolong_add: the fine grid needs even cell counts");
    if ((uintptr_t)e & 15)
        return fail(PP_EINVAL, "pp_k_prolong_add: e must be 16-byte aligned (x-pairs are vectors)");
    launch_prolong<double>(to_dims(grid), to_bc(grid), eH, e, nullptr, (hipStream_t)hip_stream);
    return check_launch("pp_k_prolong_add");
}

int pp_k_prolong_weights(const pp_grid *grid, const double *bx, const double *by,
                         const double *bz, uint32_t *w, void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!bx || !by || !bz || !w)
        return fail(PP_EINVAL, "pp_k_prolong_weights: NULL array");
    launch_prolong_weights(to_dims(grid), to_bc(grid), bx, by, bz, w, (hipStream_t)hip_stream);
    return check_launch("pp_k_prolong_weights");
}

int pp_k_prolong_add_weighted(const pp_grid *grid, const double *eH, const uint32_t *w, double *e,
                              void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!eH || !e || !w)
        return fail(PP_EINVAL, "pp_k_prolong_add_weighted: NULL array");
    for (int m = 0; m < 3; ++m)
        if (grid->n[m] % 2)
            return fail(PP_EINVAL, "pp_k_prolong_add_weighted: the fine grid needs even cell counts");
    if (((uintptr_t)e & 15) || ((uintptr_t)w & 7))
        return fail(PP_EINVAL, "pp_k_prolong_add_weighted: e must be 16-byte aligned and w "
                               "8-byte aligned (x-pairs are vectors)");
    launch_prolong<double>(to_dims(grid), to_bc(grid), eH, e, w, (hipStream_t)hip_stream);
    return check_launch("pp_k_prolong_add_weighted");
}

int pp_k_coarsen_beta(const pp_grid *grid, const double *bx, const double *by, const double *bz,
                      double *hx, double *hy, double *hz, void *hip_stream)
{
    PP_TRY(validate_grid(grid, nullptr, nullptr, nullptr));
    if (!bx || !by || !bz || !hx || !hy || !hz)
        return fail(PP_EINVAL, "pp_k_coarsen_beta: NULL array");
    for (int m = 0; m < 3; ++m)
        if (grid->n[m] % 2)
            return fail(PP_EINVAL, "pp_k_coarsen_beta: the fine grid needs even cell counts");
    launch_coarsen_beta(to_dims(grid), to_bc(grid), bx, by, bz, hx, hy, hz, (hipStream_t)hip_stream);
    return check_launch("pp_k_coarsen_beta");
}

int pp_vcycle(pp_ctx *c, const double *r, double *e)
{
    PP_TRY(check_ctx(c));
    if (!r || !e)
        return fail(PP_EINVAL, "pp_vcycle: NULL array");
    PP_TRY(ensure_pinv(c));
    Hier &H = (c->opts.precision == PP_FP64) ? c->h64 : c->hmix;
    LevelBuf &v0 = H.lev[0];
    switch (H.st) {
    case ST_F64:
        launch_copy(r, (double *)v0.r, c->N, c->stream);
        PP_TRY(vcycle_run<double>(c, H));
        launch_copy((const double *)v0.cur, e, c->N, c->stream);
        break;
    case ST_F32:
        launch_convert<float>(c->N, r, (float *)v0.r, c->stream);
        PP_TRY(vcycle_run<float>(c, H));
        launch_to_double<float>(c->N, (const float *)v0.cur, e, c->stream);
        break;
    default:
        launch_convert<_Float16>(c->N, r, (_Float16 *)v0.r, c->stream);
        PP_TRY(vcycle_run<_Float16>(c, H));
        launch_to_double<_Float16>(c->N, (const _Float16 *)v0.cur, e, c->stream);
        break;
    }
    return check_launch("pp_vcycle");
}

int pp_k_copy(const double *src, double *dst, int64_t count, void *hip_stream)
{
    if (!src || !dst || count < 0)
        return fail(PP_EINVAL, "pp_k_copy: bad arguments");
    if (count == 0)
        return PP_OK;
    launch_copy(src, dst, (size_t)count, (hipStream_t)hip_stream);
    return check_launch("pp_k_copy");
}

int pp_timing_enable(pp_ctx *c, int32_t mask)
{
    PP_TRY(check_ctx(c));
    if (mask < 0 || mask >= (1 << PP_KT_COUNT))
        return fail(PP_EINVAL, "pp_timing_enable: mask has bits beyond the kernel kinds");
    if (mask && c->ev.empty()) {
        // timing only: no system-scope fence (cache writeback) when they
        // complete, which would stall the kernels queued behind them
        c->ev.resize(8192);
        for (auto &e : c->ev) {
            PP_HIP(hipEventCreateWithFlags(&e.a, hipEventDisableSystemFence));
            PP_HIP(hipEventCreateWithFlags(&e.b, hipEventDisableSystemFence));
        }
    }
    if (!mask)
        resolve_timing(c);
    c->timing = mask != 0;
    c->timing_mask = (uint32_t)mask;
    return PP_OK;
}

int pp_timing_reset(pp_ctx *c)
{
    PP_TRY(check_ctx(c));
    resolve_timing(c);
    for (int k = 0; k < PP_KT_COUNT; ++k) {
        c->kt_count[k] = 0;
        c->kt_ms[k] = 0.0;
    }
    return PP_OK;
}

int pp_timing_get(pp_ctx *c, int32_t kind, int64_t *launches, double *total_ms)
{
    PP_TRY(check_ctx(c));
    if (kind < 0 || kind >= PP_KT_COUNT || !launches || !total_ms)
        return fail(PP_EINVAL, "pp_timing_get: bad kind or NULL output");
    resolve_timing(c);
    *launches = c->kt_count[kind];
    *total_ms = c->kt_ms[kind];
    return PP_OK;
}

}  // extern "C"
