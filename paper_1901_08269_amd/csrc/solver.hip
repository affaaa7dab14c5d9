// solver.hip -- host side of the C-ABI declared in include/cps.h: device memory, the setup
// sequence, the BiCGSTAB driver (Alg. 1) in FP64, and the FP32-inner / FP64-refinement
// driver.  Every arithmetic step runs in the kernels of setup.hip and sweeps.hip; the host
// only launches, polls one small device-state record per iteration and checks the final
// FP64 residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "cps.h"
#include "cps_device.h"
#include "cps_kernels.h"

using namespace cps;

namespace {

// Preconditioner defaults: Chebyshev-Jacobi steps per apply, and the interval [lo, hi] for
// the spectrum of diag(K)^-1 K.  hi = 2 is the Gershgorin bound of the diagonally dominant
// rows of K.  lo = 0 selects max(hi / (4 m^2), lambda_1): hi / (4 m^2) is the lower end at
// which an m-step Chebyshev polynomial still damps the smooth error (measured best to
// within a few iterations for m = 8 ... 32 on 256^3 stretched grids with bodies), and
// lambda_1 = (1/3) sum_d (1 - cos(pi / (n_d - 1))) is the smallest eigenvalue of the
// Jacobi-scaled 7-point Laplacian on a uniform grid with the same point counts, below
// which a small grid has no spectrum to cover.
constexpr int DEFAULT_INNER = 24;
constexpr double DEFAULT_LAM_HI = 2.0;
constexpr int ELL_CAP = 243;               // 27 box nodes + 216 extra-point positions
constexpr int MAX_INNER = 64;
static_assert(MAX_INNER <= MG_MAX_COARSE_STEPS, "the coarsest level's steps fit its kernel's coefficient array");

template <typename T>
struct Vecs {
    T *r = nullptr, *r0 = nullptr, *p = nullptr, *ph = nullptr, *v = nullptr, *s = nullptr, *sh = nullptr, *t = nullptr;
    T *x = nullptr, *c[2] = {nullptr, nullptr};
    bool ready = false;
};

// Multigrid preconditioner for K: a coarser level keeps the even-indexed points and the
// last one along every axis while every axis has at least 2 MG_MIN_POINTS - 1 points and
// the level has more than MG_LDS_NODES interior points (a level that small is solved in one
// workgroup).
constexpr int MG_MIN_POINTS = 9;
constexpr int MG_MAX_LEVELS = 16;

// One level of the multigrid hierarchy.  Level 0 aliases the solver's own grid data; a
// coarser level owns its coordinates, 1D tables, node types, skip bits and K rows (no B).
struct MgLevel {
    int n[3] = {0, 0, 0};
    int nmax = 0;
    size_t nn = 0;
    Geom g{};
    double *xyz = nullptr;
    double *coef64 = nullptr;
    float *coef32 = nullptr;
    int8_t *type = nullptr;
    uint32_t *skip = nullptr;
    int nirr = 0;
    int *irr_node = nullptr;
    double *k64 = nullptr;
    float *k32 = nullptr;
    int *irr_map = nullptr;     // node -> irregular row (coarse levels)
    double *dg64 = nullptr;     // diagonal of K at the unknown nodes, 0 elsewhere (coarse
    float *dg32 = nullptr;      // levels, built on first use of the precision)
    bool lds = false;           // the coarsest level, solved in one workgroup
    MgTransfer<double> t64{};   // transfers to the next coarser level
    MgTransfer<float> t32{};
    double *v64[4] = {nullptr, nullptr, nullptr, nullptr};   // level right-hand side, two iterates, residual
    float *v32[4] = {nullptr, nullptr, nullptr, nullptr};
};

}  // namespace

struct cps_solver {
    cps_options opt;
    hipStream_t stream = nullptr;
    Geom g{};
    int nx = 0, ny = 0, nz = 0, nmax = 0;
    size_t nn = 0;
    // device data
    double *xyz = nullptr;        // x | y | z
    double *coef64 = nullptr;     // 3 * 8 * nmax
    float *coef32 = nullptr;
    double *phi = nullptr, *gf = nullptr, *f = nullptr;
    int8_t *type = nullptr;
    uint32_t *skip = nullptr;
    double *dot_partials = nullptr;  // warm-start scaling: per-block partial dots
    uint32_t *irr_bits = nullptr;  // irregular-node bits (skip-word layout)
    int *irr_wstart = nullptr;     // irregular rows before each bit word
    int nirr = 0;
    int *irr_node = nullptr, *irr_ptr = nullptr, *irr_col = nullptr;
    double *irr_val64 = nullptr, *irr_k64 = nullptr, *irr_bd64 = nullptr;
    float *irr_val32 = nullptr, *irr_k32 = nullptr, *irr_bd32 = nullptr;
    double *rhs = nullptr;
    double *partials = nullptr;
    DevState *st = nullptr;
    int *dflag = nullptr;
    DevState *hst = nullptr;      // pinned, 2 slots
    double *hscalar = nullptr;    // pinned staging
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> tev;  // sweep timing events
    size_t tev_used = 0;
    int64_t sweep_count = 0;      // preconditioner applies since the solve started (timing sample)
    int64_t iter_enq = 0;         // BiCGSTAB iterations enqueued since the solve started
    std::vector<int64_t> tev_iter;  // per timed sweep: the iteration it belongs to
    std::vector<char> tev_ok;       // per timed sweep: ran (not after the solve had converged)
    std::vector<int> tev_n;         // per timed sweep: sweeps (1)
    std::vector<int> tev_vec;       // per timed sweep: vectors it reads and writes
    // residual history of the last solve: per iteration the recursive ||D^-1 r|| / ||D^-1 b||,
    // per restart pass or refinement step the true (||r||/||b||, ||D^-1 r||/||D^-1 b||)
    std::vector<double> hist_iter, hist_true;
    int hist_it0 = 0;               // DevState.iters when the current run of iterations began
    int hist_run = 0;               // iterations of the current run recorded
    Vecs<double> v64;
    Vecs<float> v32;
    double *tmp64 = nullptr;      // user-facing staging (residual, apply, precond)
    double *x64 = nullptr;        // FP64 solution in mixed mode
    float *tmp32a = nullptr, *tmp32b = nullptr;
    // multigrid preconditioner (opt.precond = CPS_PRECOND_MULTIGRID)
    std::vector<MgLevel> mg;            // mg[0] is this grid
    std::vector<double> mg_c1, mg_c2;   // smoother steps on [mg_smooth_lo, lam_hi]
    std::vector<double> mg_cc1, mg_cc2; // coarsest-level steps on [lambda_1, lam_hi]
    double *mg_zero64 = nullptr;        // zeros, the size of level 1
    float *mg_zero32 = nullptr;
    int sweep_rev[MG_MAX_LEVELS] = {};  // per level: z direction of its next sweep (alternates)
    double *mg_ccd64 = nullptr;         // mg_cc1 | mg_cc2 on the device (one-workgroup coarsest solve)
    float *mg_ccd32 = nullptr;
    // strongly implicit procedure (opt.precond = CPS_PRECOND_SIP): factors b, c, d, e, f, g, h
    // (and a zero) per node in FP64 and FP32, the irregular row of each irregular node, and
    // per precision the residual and substitution vectors
    double *sip64 = nullptr;
    float *sip32 = nullptr;
    int *sip_map = nullptr;
    double *sip_w64[2] = {nullptr, nullptr};
    float *sip_w32[2] = {nullptr, nullptr};
    // host-side facts
    long long n_unknown = 0, n_solid = 0, nnz = 0, fallback = 0;
    double min_hb = 1.0;
    double bn2 = 0.0, bs2 = 0.0;  // ||b||^2, ||D^-1 b||^2
    double setup_ms = 0.0;
    struct Alloc {
        void *p;
        size_t bytes;
    };
    std::vector<Alloc> allocs;    // device blocks owned by this solver

    Launch launch() const { return Launch{g, stream, skip, partials}; }
    Coef<double> cf64() const
    {
        Coef<double> c;
        for (int d = 0; d < 3; ++d) c.c[d] = coef64 + (size_t)d * 8 * nmax;
        return c;
    }
    Coef<float> cf32() const
    {
        Coef<float> c;
        for (int d = 0; d < 3; ++d) c.c[d] = coef32 + (size_t)d * 8 * nmax;
        return c;
    }
    Irr<double> ir64() const
    {
        return Irr<double>{nirr, irr_node, irr_ptr, irr_col, irr_val64, irr_k64, irr_bd64, irr_bits, irr_wstart};
    }
    Irr<float> ir32() const
    {
        return Irr<float>{nirr, irr_node, irr_ptr, irr_col, irr_val32, irr_k32, irr_bd32, irr_bits, irr_wstart};
    }
};

namespace {

struct HipFail {
    hipError_t e;
};

inline void ck(hipError_t e)
{
    if (e != hipSuccess) throw HipFail{e};
}

// Pinned host blocks for the small device-to-host state copies.  Freeing pinned memory is
// slow (it synchronises and unpins), so blocks go back to a process-wide free list.
constexpr size_t PINNED_BLOCK = 4096;
std::mutex pinned_mu;
std::vector<void *> pinned_free;

void *pinned_get()
{
    {
        std::lock_guard<std::mutex> lk(pinned_mu);
        if (!pinned_free.empty()) {
            void *p = pinned_free.back();
            pinned_free.pop_back();
            return p;
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, PINNED_BLOCK, hipHostMallocDefault) != hipSuccess) throw std::bad_alloc();
    return p;
}

void pinned_put(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(pinned_mu);
    pinned_free.push_back(p);
}

// Device memory cache.  Returning memory to the HIP runtime costs about a quarter of a
// millisecond per block, so blocks released by a solver (at destroy, or setup temporaries)
// stay in a per-device list and serve later allocations of up to the same size; only a
// miss allocates.  Blocks enter the list idle (the owning stream is synchronised first), so
// any stream may reuse them.  An allocation that fails releases the device's cached blocks
// and retries once.  The cache lives until the process ends.
struct CachedBlock {
    void *p;
    size_t bytes;
    int dev;
};
std::mutex cache_mu;
std::vector<CachedBlock> cache_blocks;

size_t cache_round(size_t bytes)
{
    const size_t g = bytes >= ((size_t)1 << 20) ? ((size_t)2 << 20) : 256;
    return (bytes + g - 1) / g * g;
}

void *cache_alloc(size_t bytes)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) throw std::bad_alloc();
    bytes = cache_round(bytes);
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        int best = -1;
        for (int q = 0; q < (int)cache_blocks.size(); ++q) {
            const CachedBlock &c = cache_blocks[q];
            if (c.dev == dev && c.bytes >= bytes && c.bytes <= 2 * bytes &&
                (best < 0 || c.bytes < cache_blocks[best].bytes))
                best = q;
        }
        if (best >= 0) {
            void *p = cache_blocks[best].p;
            cache_blocks.erase(cache_blocks.begin() + best);
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) == hipSuccess) return p;
    (void)hipGetLastError();
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        for (int q = (int)cache_blocks.size() - 1; q >= 0; --q)
            if (cache_blocks[q].dev == dev) {
                (void)hipFree(cache_blocks[q].p);
                cache_blocks.erase(cache_blocks.begin() + q);
            }
    }
    if (hipMalloc(&p, bytes) == hipSuccess) return p;
    (void)hipGetLastError();
    throw std::bad_alloc();
}

void cache_release(void *p, size_t bytes)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(cache_mu);
    cache_blocks.push_back(CachedBlock{p, cache_round(bytes), dev});
}

template <typename T>
T *dalloc(cps_solver *s, size_t n)
{
    if (n == 0) n = 1;
    void *p = cache_alloc(n * sizeof(T));
    s->allocs.push_back({p, n * sizeof(T)});
    return (T *)p;
}

void dfree(cps_solver *s, void *p)
{
    if (!p) return;
    auto it = std::find_if(s->allocs.begin(), s->allocs.end(), [&](const cps_solver::Alloc &a) { return a.p == p; });
    if (it == s->allocs.end()) return;
    (void)hipStreamSynchronize(s->stream);
    cache_release(it->p, it->bytes);
    s->allocs.erase(it);
}

// copy a caller array (host or device per opt.device_ptrs) to device memory
void to_device(cps_solver *s, void *dst, const void *src, size_t bytes)
{
    ck(hipMemcpyAsync(dst, src, bytes, s->opt.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
}

void from_device(cps_solver *s, void *dst, const void *src, size_t bytes)
{
    ck(hipMemcpyAsync(dst, src, bytes, s->opt.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
}

void sync(cps_solver *s) { ck(hipStreamSynchronize(s->stream)); }

DevState read_state(cps_solver *s)
{
    ck(hipMemcpyAsync(&s->hst[0], s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    sync(s);
    return s->hst[0];
}

void set_stop2(cps_solver *s, double v)
{
    // staged through pinned memory; the copy is ordered with the kernels on the stream
    s->hscalar[0] = v;
    ck(hipMemcpyAsync(&s->st->stop2, s->hscalar, sizeof(double), hipMemcpyHostToDevice, s->stream));
}

Tiling make_tiling(int nx, int ny, int nz, int tw, int ty, int target_blocks, int min_tz)
{
    Tiling t{};
    t.tw = tw;
    t.ty = ty;
    t.tiles_x = (nx - 2 + tw - 1) / tw;
    t.tiles_y = (ny - 2 + ty - 1) / ty;
    int per_plane = t.tiles_x * t.tiles_y;
    int nzi = nz - 2;
    int want = std::max(1, (target_blocks + per_plane - 1) / per_plane);
    t.TZ = std::max(std::min(min_tz, nzi), (nzi + want - 1) / want);
    t.zchunks = (nzi + t.TZ - 1) / t.TZ;
    t.ntiles = per_plane * t.zchunks;
    t.nblk = (t.ntiles + NXCD - 1) / NXCD * NXCD;
    return t;
}

// The vectorised Chebyshev sweep splits z into this many chunks (each at least 4 planes):
// measured best at 256^3 (1024 blocks, 43.0 us per FP32 sweep; 8 chunks 51.4 us, 32 chunks
// 47.5 us) and at 512^3.  Fewer chunks leave wavefronts idle; more chunks re-read more halo
// planes and put the blocks in more than one round.
constexpr int ROW_ZCHUNKS = 16;
// The FP32 two-vector sweeps (113 VGPRs, four wavefronts per SIMD, against 180 and two in
// FP64) fill the GPU with more z-chunks: 24 instead of 16 (768 instead of 512 blocks at 256^3).
constexpr int ROW_ZCHUNKS_F32 = 24;
// z-chunks of the vectorised B apply and vector updates (each at least 4 planes; 8 and 32
// measured the same at 256^3)
constexpr int APPLY_ZCHUNKS = 16;
// grid-stride kernels over all nodes (fills, copies, restart) use at most this many blocks
constexpr int FLAT_BLOCKS = 4096;

// coarse = true (a coarse multigrid level): the sweep tiling aims at COARSE_TILES tiles
// of at least one plane each, since a small grid's sweep is bound by the latency of its
// z-march rather than by bandwidth (spheres8 256^3, mixed multigrid solve: 1024 tiles
// 25.1 ms, 512 25.2 ms, 2048 25.6 ms)
constexpr int COARSE_TILES = 1024;
Geom make_geom(int nx, int ny, int nz, bool coarse = false)
{
    Geom g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.W = (nx + 31) / 32;
    {
        const int per_plane = ((nx - 2 + 4 * TX - 1) / (4 * TX)) * ((ny - 2 + TY - 1) / TY);
        g.ta = make_tiling(nx, ny, nz, 4 * TX, TY, per_plane * APPLY_ZCHUNKS, 4);
    }
    // a coarse level whose rows need at most 32 lanes packs 64 / 2^lg rows into a wavefront
    g.lg = 6;
    if (coarse && RPW == 1)
        while (g.lg > 3 && 4 * (1 << (g.lg - 1)) >= nx - 2) --g.lg;
    {
        const int per_plane = ((nx - 2 + 4 * TX - 1) / (4 * TX)) * ((ny - 2 + TY * RPW - 1) / (TY * RPW));
        g.tr = coarse ? make_tiling(nx, ny, nz, 4 << g.lg, TY * RPW * (TX >> g.lg), COARSE_TILES, 1)
                      : make_tiling(nx, ny, nz, 4 * TX, TY * RPW, per_plane * ROW_ZCHUNKS, 4);
        const int per_plane2 = ((nx - 2 + 4 * TX - 1) / (4 * TX)) * ((ny - 2 + TY * RPW2 - 1) / (TY * RPW2));
        g.tr2 = make_tiling(nx, ny, nz, 4 * TX, TY * RPW2, per_plane2 * ROW_ZCHUNKS, 4);
        g.tr2s = make_tiling(nx, ny, nz, 4 * TX, TY * RPW2, per_plane2 * ROW_ZCHUNKS_F32, 4);
    }
    size_t nn = (size_t)nx * ny * nz;
    g.nflat = (int)std::min<size_t>((nn / 4 + 255) / 256 + 1, FLAT_BLOCKS);
    return g;
}

// Chebyshev step coefficients for [lo, hi] (Saad, Alg. 12.1): c1[0] = 0, c2[0] = 1/theta
void cheb_coefficients(int m, double lo, double hi, double *c1, double *c2)
{
    double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rp = 1.0 / sigma;
    c1[0] = 0.0;
    c2[0] = 1.0 / theta;
    for (int k = 1; k < m; ++k) {
        double r = 1.0 / (2.0 * sigma - rp);
        c1[k] = r * rp;
        c2[k] = 2.0 * r / delta;
        rp = r;
    }
}

template <typename T>
void alloc_vecs(cps_solver *s, Vecs<T> &V)
{
    if (V.ready) return;
    // every kernel writes a vector's unknowns before it reads them (the Krylov vectors are set
    // by the restart, the iterates by each pass's first step), and reads the other nodes and
    // the padding as zeros: one launch zeroes those in all vectors
    T **all[] = {&V.r, &V.r0, &V.p, &V.ph, &V.v, &V.s, &V.sh, &V.t, &V.x, &V.c[0], &V.c[1]};
    VecList<T> list{};
    for (T **p : all) {
        *p = dalloc<T>(s, s->nn + VEC_PAD);
        list.p[list.n++] = *p;
    }
    launch_zero_off_unknowns<T>(s->stream, s->nn, VEC_PAD, s->type, list);
    V.ready = true;
}

hipEvent_t timing_event(cps_solver *s)
{
    if (s->tev_used == s->tev.size()) {
        hipEvent_t e;
        ck(hipEventCreate(&e));
        s->tev.push_back(e);
    }
    return s->tev[s->tev_used++];
}

// Sweep timing: every kernel_timing-th preconditioner apply is sampled (sampled_run); each of
// its sweeps on the problem's grid gets a pair of events that its launch stamps with the
// kernel's own start and end (timed_sweep), so the timing holds the sweeps' execution and no
// launch gaps or queue time.
bool sampled_run(cps_solver *s)
{
    const int period = s->opt.kernel_timing;
    return period > 0 && (s->sweep_count++ % period) == 0;
}

// events for one timed sweep that reads and writes `nvec` vectors
std::pair<hipEvent_t, hipEvent_t> timed_sweep(cps_solver *s, int nvec)
{
    hipEvent_t e0 = timing_event(s), e1 = timing_event(s);
    const size_t pair = s->tev_used / 2 - 1;
    if (s->tev_iter.size() <= pair) {
        s->tev_iter.resize(pair + 1);
        s->tev_ok.resize(pair + 1);
        s->tev_n.resize(pair + 1);
        s->tev_vec.resize(pair + 1);
    }
    s->tev_iter[pair] = s->iter_enq;
    s->tev_ok[pair] = 1;
    s->tev_n[pair] = 1;
    s->tev_vec[pair] = nvec;
    return {e0, e1};
}

// ---- multigrid V-cycle on K (the inner solver of the preconditioner, Sec. 3.3) ----------
template <typename T>
T *const *mg_vecs(const MgLevel &Lv)
{
    if constexpr (sizeof(T) == 8) return Lv.v64; else return Lv.v32;
}

template <typename T>
const MgTransfer<T> &mg_transfer(const MgLevel &Lv)
{
    if constexpr (sizeof(T) == 8) return Lv.t64; else return Lv.t32;
}

// level vectors of precision T (allocated and zeroed on first use)
template <typename T>
void mg_alloc(cps_solver *s)
{
    for (size_t l = 1; l < s->mg.size(); ++l) {
        MgLevel &Lv = s->mg[l];
        T **v;
        if constexpr (sizeof(T) == 8) v = Lv.v64; else v = Lv.v32;
        // as for the problem grid's vectors: the unknowns are written before they are read
        VecList<T> list{};
        for (int q = 0; q < 4; ++q)
            if (!v[q]) {
                v[q] = dalloc<T>(s, Lv.nn + VEC_PAD);
                list.p[list.n++] = v[q];
            }
        launch_zero_off_unknowns<T>(s->stream, Lv.nn, VEC_PAD, Lv.type, list);
    }
    if (s->mg.size() > 1) {
        T **z;
        if constexpr (sizeof(T) == 8) z = &s->mg_zero64; else z = &s->mg_zero32;
        if (!*z) {
            *z = dalloc<T>(s, s->mg[1].nn + VEC_PAD);
            launch_fill<T>(s->stream, s->mg[1].nn + VEC_PAD, *z, T(0));
        }
    }
}

template <typename T>
Coef<T> mg_coef(const MgLevel &Lv)
{
    Coef<T> c;
    for (int d = 0; d < 3; ++d) {
        if constexpr (sizeof(T) == 8) c.c[d] = Lv.coef64 + (size_t)d * 8 * Lv.nmax;
        else c.c[d] = Lv.coef32 + (size_t)d * 8 * Lv.nmax;
    }
    return c;
}

// the K rows of a coarse level (the fields of B are not used by the K sweeps)
template <typename T>
Irr<T> mg_irr(const MgLevel &Lv)
{
    Irr<T> r{};
    r.n = Lv.nirr;
    r.node = Lv.irr_node;
    if constexpr (sizeof(T) == 8) r.k7 = Lv.k64; else r.k7 = Lv.k32;
    return r;
}

// Steps k0 .. n-1 of a Chebyshev-Jacobi iteration on K x = rho (coefficients c1, c2).
// From x = 0 (x0 null; `zero` is read as x_0 when k0 = 0) the iterates alternate a, b, a, ...;
// from x0 (which must be a) they alternate b, a, b, ...  Each step from the third on writes
// over its x_{k-1} in place.  The last step writes dst if it is non-null.  Returns the
// buffer that holds x_n.  Level-0 sweeps with an x_{k-1} are sampled by kernel_timing.
// z direction of the next sweep on level l: consecutive sweeps of a level alternate, each
// starting on the planes the previous one touched last
int next_rev(cps_solver *s, int l)
{
    const int r = s->sweep_rev[l];
    s->sweep_rev[l] ^= 1;
    return r;
}

template <typename T>
T *mg_smooth(cps_solver *s, int lvl, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *rho, T *x0,
             const T *zero, T *a, T *b, T *dst, int k0, int n, const double *c1, const double *c2, const DevState *st,
             bool timed)
{
    T *odd = x0 ? b : a, *even = x0 ? a : b;
    auto buf = [&](int j) -> T * { return j == 0 ? (x0 ? x0 : (T *)zero) : ((j & 1) ? odd : even); };
    // timed: a smoothing pass on the problem's grid in a sampled cycle; each sweep reads x_k
    // and rho (and x_{k-1} except in a pass's first step) and writes x_{k+1}
    const bool sample = timed && n > k0;
    for (int k = k0; k < n; ++k) {
        const T *xm1 = (k == 0) ? nullptr : (k == 1 ? (const T *)x0 : buf(k - 1));
        T *out = (k == n - 1 && dst) ? dst : buf(k + 1);
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (sample) ev = timed_sweep(s, xm1 ? 4 : 3);
        launch_cheb<T>(L, cf, ir, buf(k), xm1, rho, out, c1[k], c2[k], st, next_rev(s, lvl), ev.first, ev.second);
    }
    return dst ? dst : buf(n);
}

// What the restriction into coarse level l needs besides rho_l: the level's diagonal (which
// marks its unknowns) and, except on the last level (whose own iteration starts from zero),
// the first iterate buffer that takes the level's first Chebyshev step from zero.
template <typename T>
MgFirst<T> mg_first(cps_solver *s, int l)
{
    MgFirst<T> f{};
    const MgLevel &Lv = s->mg[l];
    if constexpr (sizeof(T) == 8) f.diag = Lv.dg64; else f.diag = Lv.dg32;
    if (l + 1 == (int)s->mg.size()) return f;
    f.x1 = mg_vecs<T>(Lv)[1];
    f.c2 = (T)s->mg_c2[0];
    return f;
}

// smoother steps k0 .. n - 1 (at most MG_TB_H) of a coarse level's pass, for one launch
template <typename T>
MgSteps<T> mg_steps(const cps_solver *s, int k0, int n)
{
    MgSteps<T> S{};
    S.n = n - k0;
    for (int q = 0; q < S.n; ++q) {
        S.c1[q] = (T)s->mg_c1[k0 + q];
        S.c2[q] = (T)s->mg_c2[k0 + q];
    }
    return S;
}

// V-cycle on coarse level l >= 1 for K_l x = rho_l (rho_l in the level's first vector and,
// unless l is the last level, its first step x_1 in the second, both from the restriction);
// returns the buffer that holds x.
template <typename T>
T *mg_level(cps_solver *s, int l, const DevState *st)
{
    const MgLevel &Lv = s->mg[l];
    T *const *V = mg_vecs<T>(Lv);
    T *R = V[0], *A = V[1], *B = V[2];
    const T *Z;
    if constexpr (sizeof(T) == 8) Z = s->mg_zero64; else Z = s->mg_zero32;
    const Launch L{Lv.g, s->stream, Lv.skip, s->partials};
    const Coef<T> cf = mg_coef<T>(Lv);
    const Irr<T> ir = mg_irr<T>(Lv);
    if (l + 1 == (int)s->mg.size()) {
        if (Lv.lds) {
            const T *cc;
            if constexpr (sizeof(T) == 8) cc = s->mg_ccd64; else cc = s->mg_ccd32;
            launch_mg_coarsest<T>(s->stream, Lv.n[0], Lv.n[1], Lv.n[2], cf, Lv.type, Lv.irr_map, ir.k7, R, A,
                                  s->opt.mg_coarse_steps, cc, cc + s->mg_cc1.size(), st);
            return A;
        }
        return mg_smooth<T>(s, l, L, cf, ir, R, nullptr, Z, A, B, nullptr, 0, s->opt.mg_coarse_steps, s->mg_cc1.data(),
                            s->mg_cc2.data(), st, false);
    }
    const int nu = s->opt.mg_nu;
    if (nu <= MG_TB_H && (long long)(Lv.n[0] - 2) * (Lv.n[1] - 2) * (Lv.n[2] - 2) <= MG_TB_MAX_POINTS) {
        // each smoothing pass in one temporally blocked launch: steps 1 .. nu - 1 from the
        // restriction's first step x_1 (in A), then the residual restricted into the next
        // level in the same launch (or, for more steps than that leaves room for, stored
        // and restricted apart); after the coarse correction, steps 0 .. nu - 1 from the
        // iterate with the prolonged correction added on load
        const MgTransfer<T> &tr = mg_transfer<T>(Lv);
        const MgFirst<T> first = mg_first<T>(s, l + 1);
        T *rc = mg_vecs<T>(s->mg[l + 1])[0];
        if (nu - 1 <= MG_TB_H - 2) {
            launch_mg_smooth_tb<T>(s->stream, Lv.n[0], Lv.n[1], Lv.n[2], cf, Lv.type, Lv.irr_map, ir.k7, R, A, B,
                                   nullptr, mg_steps<T>(s, 1, nu), st, &tr, nullptr, rc, &first);
        } else {
            T *Rr = V[3];
            launch_mg_smooth_tb<T>(s->stream, Lv.n[0], Lv.n[1], Lv.n[2], cf, Lv.type, Lv.irr_map, ir.k7, R, A, B, Rr,
                                   mg_steps<T>(s, 1, nu), st);
            launch_mg_restrict<T>(s->stream, tr, Rr, rc, first);
        }
        T *e = mg_level<T>(s, l + 1, st);
        launch_mg_smooth_tb<T>(s->stream, Lv.n[0], Lv.n[1], Lv.n[2], cf, Lv.type, Lv.irr_map, ir.k7, R, B, A, nullptr,
                               mg_steps<T>(s, 0, nu), st, &tr, e);
        return A;
    }
    T *x = mg_smooth<T>(s, l, L, cf, ir, R, nullptr, Z, A, B, nullptr, 1, nu, s->mg_c1.data(), s->mg_c2.data(), st, false);
    T *r = (x == A) ? B : A;
    launch_resid<T>(L, cf, ir, x, R, r, st, next_rev(s, l));
    launch_mg_restrict<T>(s->stream, mg_transfer<T>(Lv), r, mg_vecs<T>(s->mg[l + 1])[0], mg_first<T>(s, l + 1));
    T *e = mg_level<T>(s, l + 1, st);
    launch_mg_prolong_add<T>(s->stream, mg_transfer<T>(Lv), Lv.skip, Lv.g.W, e, x);
    return mg_smooth<T>(s, l, L, cf, ir, R, x, Z, x, r, nullptr, 0, nu, s->mg_c1.data(), s->mg_c2.data(), st, false);
}

// dst = one V-cycle for K dst = ps on the problem's grid.  The first pre-smoothing step is
// fused with the vector update `kind` that forms ps (as in the Chebyshev preconditioner);
// the iterates use the two Chebyshev buffers of V.
template <typename T>
void mg_precond(cps_solver *s, Vecs<T> &V, int kind, const T *r, T *ps, const T *v, T *dst, const DevState *st)
{
    mg_alloc<T>(s);
    for (size_t l = 1; l < s->mg.size(); ++l) {
        MgLevel &Lv = s->mg[l];
        T **dg;
        if constexpr (sizeof(T) == 8) dg = &Lv.dg64; else dg = &Lv.dg32;
        if (!*dg) {
            *dg = dalloc<T>(s, Lv.nn);
            launch_mg_diag<T>(s->stream, Lv.n[0], Lv.n[1], Lv.n[2], mg_coef<T>(Lv), Lv.type, Lv.irr_map,
                              mg_irr<T>(Lv).k7, *dg);
        }
    }
    const Launch L = s->launch();
    Coef<T> cf;
    Irr<T> ir;
    if constexpr (sizeof(T) == 8) { cf = s->cf64(); ir = s->ir64(); } else { cf = s->cf32(); ir = s->ir32(); }
    T *a = V.c[1], *b = V.c[0];
    // every kernel_timing-th cycle times both smoothing passes on this grid (sampling single
    // passes would alias with the two passes of a cycle)
    const bool samp = sampled_run(s);
    if (s->mg.size() == 1) {   // no coarser grid: the coarsest-level iteration on this grid
        launch_first<T>(kind, L, cf, ir, r, ps, v, a, s->mg_cc2[0], st);
        mg_smooth<T>(s, 0, L, cf, ir, ps, nullptr, nullptr, a, b, dst, 1, s->opt.mg_coarse_steps, s->mg_cc1.data(),
                     s->mg_cc2.data(), st, samp);
        return;
    }
    const int nu = s->opt.mg_nu;
    launch_first<T>(kind, L, cf, ir, r, ps, v, a, s->mg_c2[0], st);
    T *x = mg_smooth<T>(s, 0, L, cf, ir, ps, nullptr, nullptr, a, b, nullptr, 1, nu, s->mg_c1.data(), s->mg_c2.data(), st,
                        samp);
    // the residual goes straight into the coarse right-hand side; the other buffer (0 at
    // the solid nodes, like every iterate) first takes the residual at the irregular nodes,
    // then serves as the post-smoothing's second iterate
    T *res = (x == a) ? b : a;
    launch_resid_irregular<T>(L, cf, ir, x, ps, res, st);
    launch_mg_resid_restrict<T>(s->stream, s->g, cf, L.skip, x, ps, res, mg_transfer<T>(s->mg[0]),
                                mg_vecs<T>(s->mg[1])[0], mg_first<T>(s, 1), st);
    T *e = mg_level<T>(s, 1, st);
    launch_mg_prolong_add<T>(s->stream, mg_transfer<T>(s->mg[0]), s->skip, s->g.W, e, x);
    mg_smooth<T>(s, 0, L, cf, ir, ps, x, nullptr, x, res, dst, 0, nu, s->mg_c1.data(), s->mg_c2.data(), st, samp);
}

// phi (dst) = sip_iters iterations of the strongly implicit procedure on K phi = ps from 0
template <typename T>
void sip_precond(cps_solver *s, const T *ps, T *dst, const DevState *st)
{
    T **w;
    const T *F;
    if constexpr (sizeof(T) == 8) { w = s->sip_w64; F = s->sip64; } else { w = s->sip_w32; F = s->sip32; }
    for (int q = 0; q < 2; ++q)
        if (!w[q]) {
            w[q] = dalloc<T>(s, s->nn + VEC_PAD);
            launch_fill<T>(s->stream, s->nn + VEC_PAD, w[q], T(0));
        }
    const Launch L = s->launch();
    Coef<T> cf;
    Irr<T> ir;
    if constexpr (sizeof(T) == 8) { cf = s->cf64(); ir = s->ir64(); } else { cf = s->cf32(); ir = s->ir32(); }
    for (int it = 0; it < s->opt.sip_iters; ++it) {
        const T *rin = ps;
        if (it > 0) {
            launch_resid<T>(L, cf, ir, dst, ps, w[0], st, next_rev(s, 0));
            rin = w[0];
        }
        launch_sip_iteration<T>(s->stream, s->nx, s->ny, s->nz, s->type, F, rin, w[1], dst, it == 0, st);
    }
}

// factors of the strongly implicit procedure (setup)
void sip_build(cps_solver *s)
{
    s->sip_map = dalloc<int>(s, s->nn);
    launch_mg_irr_map(s->stream, s->nirr, s->irr_node, s->sip_map);
    s->sip64 = dalloc<double>(s, 8 * s->nn);
    s->sip32 = dalloc<float>(s, 8 * s->nn);
    launch_fill<double>(s->stream, 8 * s->nn, s->sip64, 0.0);
    launch_fill<float>(s->stream, 8 * s->nn, s->sip32, 0.0f);
    launch_sip_factor(s->stream, s->nx, s->ny, s->nz, s->cf64(), s->type, s->sip_map, s->irr_k64, s->opt.sip_alpha,
                      s->sip64, s->sip32);
}

// p^ = M p: inner_iters Chebyshev steps.  The first is fused with the vector update `kind`
// (x_1 is pointwise from x_0 = 0); the rest are single sweeps in which x_{k+1} overwrites
// x_{k-1} in place (each node's x_{k-1} is read only by the thread that writes its x_{k+1}),
// so the iterates rotate through two buffers and one step touches three vectors (x_{k-1},
// x_k and rho); x_m goes to dst.  A sweep fusing two steps (20 instead of 32 bytes per node
// and pair) measured slower on MI355X (114 us per pair against 2 x 47 us for single sweeps at
// 256^3, before the in-place rotation) and could not run in place, so it was removed.
template <typename T>
void precond_apply(cps_solver *s, Vecs<T> &V, int kind, const T *r, T *ps, const T *v, T *dst, const double *c1,
                   const double *c2, const DevState *st)
{
    if (s->opt.precond == CPS_PRECOND_MULTIGRID) {
        mg_precond<T>(s, V, kind, r, ps, v, dst, st);
        return;
    }
    if (s->opt.precond == CPS_PRECOND_SIP) {
        // the vector update that forms ps (its fused first Chebyshev step lands, unused, in a
        // rotating buffer), then the strongly implicit iterations
        Coef<T> cf;
        Irr<T> ir;
        if constexpr (sizeof(T) == 8) { cf = s->cf64(); ir = s->ir64(); } else { cf = s->cf32(); ir = s->ir32(); }
        launch_first<T>(kind, s->launch(), cf, ir, r, ps, v, V.c[0], 0.0, st);
        sip_precond<T>(s, ps, dst, st);
        return;
    }
    const Launch L = s->launch();
    Coef<T> cf;
    Irr<T> ir;
    if constexpr (sizeof(T) == 8) { cf = s->cf64(); ir = s->ir64(); } else { cf = s->cf32(); ir = s->ir32(); }
    const int m = s->opt.inner_iters;
    auto buf = [&](int j) { return (j == m) ? dst : V.c[j % 2]; };
    launch_first<T>(kind, L, cf, ir, r, ps, v, buf(1), c2[0], st);
    const bool sample = m > 1 && sampled_run(s);     // step 1 reads x_1 and p; 2 .. m-1 also x_{k-1}
    for (int k = 1; k < m; ++k) {
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (sample) ev = timed_sweep(s, k >= 2 ? 4 : 3);
        launch_cheb<T>(L, cf, ir, buf(k), (k == 1) ? nullptr : buf(k - 1), ps, buf(k + 1), c1[k], c2[k], st,
                       next_rev(s, 0), ev.first, ev.second);
    }
}

// one BiCGSTAB iteration (Alg. 1) entirely on the device
template <typename T, typename TXS>
void enqueue_iteration(cps_solver *s, Vecs<T> &V, TXS *xsol, const double *c1, const double *c2)
{
    const Launch L = s->launch();
    Coef<T> cf;
    Irr<T> ir;
    if constexpr (sizeof(T) == 8) { cf = s->cf64(); ir = s->ir64(); } else { cf = s->cf32(); ir = s->ir32(); }
    precond_apply<T>(s, V, FIRST_P, V.r, V.p, V.v, V.ph, c1, c2, s->st);        // p update; K p^ = p
    launch_apply<T, T>(MODE_V, L, cf, ir, V.ph, V.v, V.r0, nullptr, s->st);    // v = B p^; alpha
    precond_apply<T>(s, V, FIRST_S, V.r, V.s, V.v, V.sh, c1, c2, s->st);       // s = r - alpha v; K s^ = s
    launch_apply<T, T>(MODE_T, L, cf, ir, V.sh, V.t, V.s, nullptr, s->st);     // t = B s^; omega
    launch_update<T, TXS>(L, cf, ir, xsol, V.ph, V.sh, V.s, V.t, V.r0, V.r, s->st);  // x, r, beta
}

// Residual history: record the recursive residual of every iteration of the current run
// that the state h has completed (each iteration's state is read once it is done; an
// iteration whose state was never read, which the polling below does not produce, would
// be recorded as NaN).
void note_state(cps_solver *s, const DevState &h)
{
    const int k = h.iters - s->hist_it0;
    const double bs = s->bs2 > 0.0 ? s->bs2 : 1.0;
    for (; s->hist_run < k; ++s->hist_run)
        s->hist_iter.push_back(s->hist_run == k - 1 ? std::sqrt(h.rn2s / bs) : std::nan(""));
}

void note_true(cps_solver *s, const DevState &d)
{
    s->hist_true.push_back(std::sqrt(d.res2 / (s->bn2 > 0.0 ? s->bn2 : 1.0)));
    s->hist_true.push_back(std::sqrt(d.res2s / (s->bs2 > 0.0 ? s->bs2 : 1.0)));
}

// run iterations until the device reports done or `budget` iterations were enqueued;
// the host polls the state of iteration n-1 while iteration n is queued.
template <typename T, typename TXS>
DevState run_iterations_enqueue(cps_solver *s, Vecs<T> &V, TXS *xsol, int budget, const double *c1, const double *c2)
{
    // Iteration n is queued before the state of iteration n - 1 is read back, so the GPU
    // does not wait for the host.  An iteration queued after the converged one still costs
    // its launches (each kernel returns at once: about 0.25 ms at 256^3 with the multigrid
    // preconditioner), so when the last two residuals predict that iteration n converges,
    // its state is read before n + 1 is queued: a wrong prediction costs a short idle gap.
    double r1 = -1.0, r2 = -1.0;    // rn2s of the last two iterations read, r1 the later
    for (int n = 0; n < budget; ++n) {
        enqueue_iteration<T, TXS>(s, V, xsol, c1, c2);
        ++s->iter_enq;
        ck(hipMemcpyAsync(&s->hst[n & 1], s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
        ck(hipEventRecord(s->ev[n & 1], s->stream));
        if (n >= 1) {
            ck(hipEventSynchronize(s->ev[(n - 1) & 1]));
            const DevState &h = s->hst[(n - 1) & 1];
            note_state(s, h);
            if (h.done) break;
            r2 = r1;
            r1 = h.rn2s;
            // predicted rn2s of iteration n: r1 times the last reduction factor (at most 1),
            // within a factor 16 of the threshold
            if (r2 > 0.0 && r1 * std::min(1.0, r1 / r2) <= 16.0 * h.stop2) {
                ck(hipEventSynchronize(s->ev[n & 1]));
                note_state(s, s->hst[n & 1]);
                if (s->hst[n & 1].done) break;
            }
        }
    }
    return read_state(s);
}

// it0: the device's iteration count when the run starts (the caller knows it from the
// state it read last; a restart does not change it)
template <typename T, typename TXS>
DevState run_iterations(cps_solver *s, Vecs<T> &V, TXS *xsol, int budget, const double *c1, const double *c2,
                        int it0)
{
    const int64_t base = s->iter_enq;
    s->hist_it0 = it0;
    s->hist_run = 0;
    DevState out = run_iterations_enqueue<T, TXS>(s, V, xsol, budget, c1, c2);
    note_state(s, out);
    // the iterations queued after the converged one return at once: their timed sweeps are
    // left out of the sweep timing
    const int64_t done = base + (out.iters - it0);
    for (size_t p = 0; p < s->tev_iter.size() && 2 * p + 1 < s->tev_used; ++p)
        if (s->tev_iter[p] >= done && s->tev_iter[p] < s->iter_enq) s->tev_ok[p] = 0;
    return out;
}

void free_solver(cps_solver *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (const auto &a : s->allocs) cache_release(a.p, a.bytes);
    s->allocs.clear();
    pinned_put(s->hst);            // hscalar lives in the same block
    for (auto &e : s->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto e : s->tev) (void)hipEventDestroy(e);
    delete s;
}

// A warm start u0 whose residual exceeds that of a zero start, ||b - B u0||_2 > ||b||_2
// (rows as stored), is scaled by the alpha that minimises ||b - alpha B u0||_2, so the start
// is never worse than zero in that norm: a coarse-grid prediction can be close to the
// solution and still have a residual far above ||b|| where the scheme's irregular rows carry
// large one-sided weights.  A start at least as good as zero is kept (alpha = 1).  Returns
// alpha.
double scale_warm_start(cps_solver *s, double *x64)
{
    const Launch L = s->launch();
    if (!s->tmp64) s->tmp64 = dalloc<double>(s, s->nn);
    double *y = s->tmp64;    // B u0 at the unknown rows
    launch_apply<double, double>(MODE_PLAIN, L, s->cf64(), s->ir64(), x64, y, nullptr, nullptr, nullptr);
    if (!s->dot_partials) s->dot_partials = dalloc<double>(s, 2 * DOT_BLOCKS);
    launch_dot2_unknowns(s->stream, s->nn, s->type, s->rhs, y, s->dot_partials);
    std::vector<double> h(2 * DOT_BLOCKS);
    ck(hipMemcpyAsync(h.data(), s->dot_partials, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    sync(s);
    double by = 0.0, yy = 0.0;
    for (int q = 0; q < DOT_BLOCKS; ++q) {
        by += h[2 * q];
        yy += h[2 * q + 1];
    }
    const double r2 = s->bn2 - 2.0 * by + yy;           // ||b - B u0||^2
    double alpha = 1.0;
    if (!(r2 <= s->bn2)) alpha = (yy > 0.0 && by > 0.0) ? by / yy : 0.0;
    if (!(alpha == alpha)) alpha = 0.0;
    if (alpha != 1.0) launch_scale(s->stream, s->nn, x64, alpha);
    return alpha;
}

int fill_stats(cps_solver *s, cps_stats *st, const DevState &ds, int iters, int iters32, int refine, int restarts,
               int status, double solve_ms)
{
    if (!st) return status;
    if (st->struct_size != (int32_t)sizeof(cps_stats) && st->struct_size != 0) return CPS_EINVAL;
    std::memset(st, 0, sizeof(*st));
    st->struct_size = sizeof(cps_stats);
    st->iters = iters;
    st->iters_fp32 = iters32;
    st->refine_steps = refine;
    st->restarts = restarts;
    st->status = status;
    st->n_unknowns = s->n_unknown;
    st->n_irregular = s->nirr;
    st->n_solid = s->n_solid;
    st->nnz_irregular = s->nnz;
    st->fallback_lines = s->fallback;
    st->rel_residual = std::sqrt(ds.res2 / (s->bn2 > 0 ? s->bn2 : 1.0));
    st->rel_residual_jacobi = std::sqrt(ds.res2s / (s->bs2 > 0 ? s->bs2 : 1.0));
    st->min_ibi_frac = s->min_hb;
    st->setup_ms = s->setup_ms;
    st->solve_ms = solve_ms;
    st->sweep_points = (int64_t)(s->nx - 2) * (s->ny - 2) * (s->nz - 2);
    if (s->opt.kernel_timing && s->tev_used >= 2) {
        double tot = 0.0, full = 0.0;
        int64_t n = 0, nvec = 0, nfull = 0;
        for (size_t q = 0; q + 1 < s->tev_used; q += 2) {
            float ms = 0.f;
            if (!s->tev_ok[q / 2]) continue;     // sweeps queued after convergence return at once
            if (hipEventElapsedTime(&ms, s->tev[q], s->tev[q + 1]) == hipSuccess) {
                tot += ms;
                n += s->tev_n[q / 2];
                nvec += s->tev_vec[q / 2];
                if (s->tev_vec[q / 2] == 4) {
                    full += ms;
                    ++nfull;
                }
            }
        }
        st->sweep_ms = tot;
        st->sweep_launches = n;
        st->sweep_full_ms = full;
        st->sweep_full_launches = nfull;
        const int vb = (s->opt.precision == CPS_MIXED) ? 4 : 8;
        st->sweep_bytes = (double)nvec * vb * (double)st->sweep_points;
    }
    return status;
}

// The irregular rows' construction in flight: its scratch buffers, between the launches
// (rows_launch) and the host's reading of their results (rows_finish).
struct RowsPending {
    int *ell_col, *len, *fb;
    double *ell_val, *rhs_row, *minhb, *ibi_tab;
};

// Queues the irregular rows (FP64) into ELL scratch and their row pointers; touches no host
// staging, so other work may use it until rows_finish.
RowsPending rows_launch(cps_solver *s)
{
    const hipStream_t st = s->stream;
    const int n = s->nirr;
    RowsPending p;
    p.ell_col = dalloc<int>(s, (size_t)n * ELL_CAP);
    p.ell_val = dalloc<double>(s, (size_t)n * ELL_CAP);
    p.len = dalloc<int>(s, n + 1);
    p.rhs_row = dalloc<double>(s, n);
    p.minhb = dalloc<double>(s, n);
    p.fb = dalloc<int>(s, n);
    if (!s->irr_k64) {
        s->irr_k64 = dalloc<double>(s, (size_t)7 * n);
        s->irr_bd64 = dalloc<double>(s, n);
        s->irr_ptr = dalloc<int>(s, n + 1);
    }
    if (!s->irr_k32) {
        s->irr_k32 = dalloc<float>(s, (size_t)7 * n);
        s->irr_bd32 = dalloc<float>(s, n);
    }
    p.ibi_tab = dalloc<double>(s, 12 * (size_t)n + 1);
    ck(hipMemsetAsync(s->dflag, 0, sizeof(int), st));
    launch_build_rows(st, s->nx, s->ny, s->nz, s->xyz, s->xyz + s->nx, s->xyz + s->nx + s->ny, s->coef64, s->phi, s->gf,
                      s->f, s->type, n, s->irr_node, s->irr_bits, s->irr_wstart, p.ibi_tab, ELL_CAP, p.ell_col,
                      p.ell_val, p.len, p.rhs_row, s->irr_k64, s->irr_bd64, p.minhb, p.fb, s->dflag);
    launch_scan(st, p.len, s->irr_ptr, n);
    return p;
}

// The rest of the right-hand side once the rows are queued: CSR packing, K rows in FP32,
// the regular and irregular right-hand side, the wall-distance and fallback summaries, the
// norms of b.
int rows_finish(cps_solver *s, const RowsPending &p)
{
    const hipStream_t st = s->stream;
    const int n = s->nirr;
    int *ell_col = p.ell_col, *len = p.len, *fb = p.fb;
    double *ell_val = p.ell_val, *rhs_row = p.rhs_row, *minhb = p.minhb, *ibi_tab = p.ibi_tab;
    int total = 0, bad = 0;
    ck(hipMemcpyAsync(s->hscalar, s->irr_ptr + n, sizeof(int), hipMemcpyDeviceToHost, st));
    ck(hipMemcpyAsync(s->hscalar + 1, s->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    sync(s);
    std::memcpy(&total, s->hscalar, sizeof(int));
    std::memcpy(&bad, s->hscalar + 1, sizeof(int));
    if (bad) {
        for (void *q : {(void *)ell_col, (void *)ell_val, (void *)len, (void *)rhs_row, (void *)minhb, (void *)fb,
                        (void *)ibi_tab})
            dfree(s, q);
        return CPS_EGEOM;   // a singular one-sided system
    }
    if (!s->irr_col || s->nnz != total) {
        dfree(s, s->irr_col);
        dfree(s, s->irr_val64);
        dfree(s, s->irr_val32);
        s->irr_col = dalloc<int>(s, total);
        s->irr_val64 = dalloc<double>(s, total);
        s->irr_val32 = dalloc<float>(s, total);
    }
    s->nnz = total;
    launch_pack_rows(st, n, ELL_CAP, ell_col, ell_val, len, s->irr_ptr, s->irr_col, s->irr_val64, s->irr_val32);
    launch_to_float(st, (size_t)7 * n, s->irr_k64, s->irr_k32);
    launch_to_float(st, (size_t)n, s->irr_bd64, s->irr_bd32);
    launch_fill<double>(st, s->nn + VEC_PAD, s->rhs, 0.0);
    launch_rhs_regular(st, s->nx, s->ny, s->nz, s->coef64, s->f, s->gf, s->type, s->rhs);
    launch_scatter_rows(st, n, s->irr_node, rhs_row, s->rhs);
    long long *dsum = dalloc<long long>(s, 1);
    double *dmin = dalloc<double>(s, 1);
    double *mpart = dalloc<double>(s, 2 * MINR_PARTS);
    if (n > 0) {
        launch_min_reduce(st, n, minhb, fb, mpart, dmin, dsum);
        ck(hipMemcpyAsync(s->hscalar, dmin, sizeof(double), hipMemcpyDeviceToHost, st));
        ck(hipMemcpyAsync(s->hscalar + 1, dsum, sizeof(long long), hipMemcpyDeviceToHost, st));
        sync(s);
        s->min_hb = s->hscalar[0];
        long long fbs;
        std::memcpy(&fbs, s->hscalar + 1, sizeof(long long));
        s->fallback = fbs;
    }
    // ||b||^2 and ||D^-1 b||^2 over the unknowns, summed on the host in block order
    if (!s->dot_partials) s->dot_partials = dalloc<double>(s, 2 * DOT_BLOCKS);
    launch_bnorms(st, s->nx, s->ny, s->nz, s->coef64, s->type, s->rhs, n, s->irr_node, s->irr_bd64, s->dot_partials,
                  DOT_BLOCKS);
    std::vector<double> hp(2 * DOT_BLOCKS);
    ck(hipMemcpyAsync(hp.data(), s->dot_partials, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    sync(s);
    s->bn2 = 0.0;
    s->bs2 = 0.0;
    for (int q = 0; q < DOT_BLOCKS; ++q) {
        s->bn2 += hp[2 * q];
        s->bs2 += hp[2 * q + 1];
    }
    for (void *q : {(void *)ell_col, (void *)ell_val, (void *)len, (void *)rhs_row, (void *)minhb, (void *)fb,
                    (void *)dsum, (void *)dmin, (void *)mpart, (void *)ibi_tab})
        dfree(s, q);
    return CPS_OK;
}

// irregular rows (FP64): ELL scratch -> CSR; K rows; diagonal; RHS; then regular RHS
int rhs_build(cps_solver *s)
{
    return rows_finish(s, rows_launch(s));
}

int count_nodes(cps_solver *s, size_t nn, const int8_t *type, int8_t want, int *list, long long *count)
{
    int nb = compact_blocks(nn);
    int *bc = dalloc<int>(s, 2 * (size_t)nb + 1);
    int *dcount = dalloc<int>(s, 1);
    int *lst = list ? list : dalloc<int>(s, nn);
    launch_compact(s->stream, nn, type, want, bc, lst, dcount, nb);
    ck(hipMemcpyAsync(s->hscalar, dcount, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    sync(s);
    int c;
    std::memcpy(&c, s->hscalar, sizeof(int));
    *count = c;
    dfree(s, bc);
    dfree(s, dcount);
    if (!list) dfree(s, lst);
    return CPS_OK;
}

int count_type(cps_solver *s, int8_t want, int *list, long long *count)
{
    return count_nodes(s, s->nn, s->type, want, list, count);
}

// A second stream per device on which the setup builds the multigrid hierarchy while the
// problem grid's irregular rows are built on the solver's stream.  Created on first use and
// kept for the process's lifetime; default priority, and non-blocking so that it also runs
// beside the null stream.
hipStream_t setup_aux_stream()
{
    static std::mutex mu;
    static std::vector<hipStream_t> per_dev;
    int dev = 0;
    ck(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if ((int)per_dev.size() <= dev) per_dev.resize(dev + 1, nullptr);
    if (!per_dev[dev]) ck(hipStreamCreateWithFlags(&per_dev[dev], hipStreamNonBlocking));
    return per_dev[dev];
}

// 1D multigrid tables of one axis: fine coordinates xf[nf], the coarse points' indices idx
// (2I for every coarse point I but the last).  Prolongation: the left coarse index a (the
// last one at most nc - 2) and the weight of coarse point a + 1 from the physical
// coordinates.  Restriction: P^T, each interior coarse row divided by its sum; its nonzero
// entries lie on fine points 2I - 1 .. 2I + 1, stored at rw[3I + (i - 2I + 1)].
void mg_axis_tables(const double *xf, int nf, const std::vector<int> &idx, std::vector<int> &pa,
                    std::vector<double> &pw, std::vector<double> &rw)
{
    const int nc = (int)idx.size();
    pa.assign(nf, 0);
    pw.assign(nf, 0.0);
    int a = 0;
    for (int i = 0; i < nf; ++i) {
        while (a + 1 <= nc - 2 && idx[a + 1] <= i) ++a;
        pa[i] = a;
        if (a != std::min(i / 2, nc - 2)) throw CPS_EINVAL;   // the kernels derive a from i
        pw[i] = (xf[i] - xf[idx[a]]) / (xf[idx[a + 1]] - xf[idx[a]]);
    }
    rw.assign(3 * (size_t)nc, 0.0);
    std::vector<double> sum(nc, 0.0);
    auto add = [&](int I, int i, double w) {
        if (w == 0.0 || I == 0 || I == nc - 1) return;   // wall rows are never restricted to
        const int q = i - (2 * I - 1);
        if (q < 0 || q > 2) throw CPS_EINVAL;
        rw[3 * I + q] += w;
        sum[I] += w;
    };
    for (int i = 0; i < nf; ++i) {
        add(pa[i], i, 1.0 - pw[i]);
        add(pa[i] + 1, i, pw[i]);
    }
    for (int I = 1; I < nc - 1; ++I)
        for (int q = 0; q < 3; ++q) rw[3 * I + q] /= sum[I];
}

// Device copy of a small host table.  The copy is asynchronous, so its source is first moved
// into `keep`, which the caller holds until the stream has been synchronised.
template <typename D>
D *upload(cps_solver *s, const std::vector<D> &h, std::vector<std::vector<char>> &keep)
{
    keep.emplace_back(reinterpret_cast<const char *>(h.data()), reinterpret_cast<const char *>(h.data() + h.size()));
    D *d = dalloc<D>(s, h.size());
    ck(hipMemcpyAsync(d, keep.back().data(), h.size() * sizeof(D), hipMemcpyHostToDevice, s->stream));
    return d;
}

// Host tables gathered into one buffer (each 256-byte aligned) and uploaded by one copy: a
// copy from pageable host memory costs the host several microseconds whatever its size.
struct Staging {
    std::vector<char> buf;
    template <typename D>
    size_t add(const std::vector<D> &h)
    {
        const size_t off = (buf.size() + 255) & ~(size_t)255;
        buf.resize(off + h.size() * sizeof(D));
        if (!h.empty()) std::memcpy(buf.data() + off, h.data(), h.size() * sizeof(D));
        return off;
    }
    char *flush(cps_solver *s, std::vector<std::vector<char>> &keep)
    {
        keep.push_back(std::move(buf));
        buf.clear();
        char *d = dalloc<char>(s, keep.back().size());
        ck(hipMemcpyAsync(d, keep.back().data(), keep.back().size(), hipMemcpyHostToDevice, s->stream));
        return d;
    }
};

// The multigrid hierarchy below the problem's grid (coordinates hx = x | y | z on the host),
// and the smoother and coarsest-level Chebyshev coefficients.
void mg_build(cps_solver *s, const std::vector<double> &hx0)
{
    s->mg.clear();
    s->mg.reserve(MG_MAX_LEVELS);
    {
        MgLevel L0;
        L0.n[0] = s->nx; L0.n[1] = s->ny; L0.n[2] = s->nz;
        L0.nmax = s->nmax;
        L0.nn = s->nn;
        L0.g = s->g;
        L0.xyz = s->xyz;
        L0.coef64 = s->coef64;
        L0.coef32 = s->coef32;
        L0.type = s->type;
        L0.skip = s->skip;
        L0.nirr = s->nirr;
        L0.irr_node = s->irr_node;
        L0.k64 = s->irr_k64;
        L0.k32 = s->irr_k32;
        s->mg.push_back(L0);
    }
    std::vector<double> hx = hx0;
    const double *phi_f = s->phi;
    std::vector<void *> temps;
    // the coarse classifications' flags (never read) go to a word of their own: the problem
    // grid's rows may be under construction on another stream, reporting into s->dflag
    int *cflag = dalloc<int>(s, 1);
    temps.push_back(cflag);
    std::vector<std::vector<char>> keep;   // sources of the asynchronous table uploads
    struct SyncFirst {                     // destroyed before `keep`, also when a step throws
        hipStream_t st;
        ~SyncFirst() { (void)hipStreamSynchronize(st); }
    } sync_first{s->stream};
    while ((int)s->mg.size() < s->opt.mg_levels) {
        MgLevel &F = s->mg.back();
        if (std::min({F.n[0], F.n[1], F.n[2]}) < 2 * MG_MIN_POINTS - 1) break;
        if ((size_t)(F.n[0] - 2) * (F.n[1] - 2) * (F.n[2] - 2) <= (size_t)MG_LDS_NODES) break;
        MgLevel C;
        std::vector<int> idx[3], gidx;
        std::vector<double> hc;
        size_t off = 0;
        // the level's host tables (transfer weights of every axis, coordinates, gather
        // indices) go up in one copy
        Staging stg;
        size_t o_pw[3], o_rw[3], o_pw32[3], o_rw32[3];
        for (int d = 0; d < 3; ++d) {
            for (int i = 0; i < F.n[d] - 1; i += 2) idx[d].push_back(i);
            if (idx[d].back() != F.n[d] - 1) idx[d].push_back(F.n[d] - 1);
            C.n[d] = (int)idx[d].size();
            for (int i : idx[d]) {
                hc.push_back(hx[off + i]);
                gidx.push_back(i);
            }
            std::vector<int> pa;
            std::vector<double> pw, rw;
            mg_axis_tables(hx.data() + off, F.n[d], idx[d], pa, pw, rw);
            pw.resize(pw.size() + 4, 0.0);   // padding: 4-vector loads of the weights
            std::vector<float> pw32(pw.begin(), pw.end()), rw32(rw.begin(), rw.end());
            o_pw[d] = stg.add(pw);
            o_rw[d] = stg.add(rw);
            o_pw32[d] = stg.add(pw32);
            o_rw32[d] = stg.add(rw32);
            F.t64.nf[d] = F.t32.nf[d] = F.n[d];
            F.t64.nc[d] = F.t32.nc[d] = C.n[d];
            off += F.n[d];
        }
        const size_t o_xyz = stg.add(hc), o_g = stg.add(gidx);
        char *dev = stg.flush(s, keep);
        for (int d = 0; d < 3; ++d) {
            F.t64.ax[d] = MgAxis<double>{(const double *)(dev + o_pw[d]), (const double *)(dev + o_rw[d])};
            F.t32.ax[d] = MgAxis<float>{(const float *)(dev + o_pw32[d]), (const float *)(dev + o_rw32[d])};
        }
        const int cx = C.n[0], cy = C.n[1], cz = C.n[2];
        C.nmax = std::max({cx, cy, cz});
        C.nn = (size_t)cx * cy * cz;
        C.g = make_geom(cx, cy, cz, true);
        C.xyz = (double *)(dev + o_xyz);
        const int *dg = (const int *)(dev + o_g);
        double *phic = dalloc<double>(s, C.nn);
        temps.push_back(phic);
        launch_gather3(s->stream, cx, cy, cz, F.n[0], F.n[1], dg, dg + cx, dg + cx + cy, phi_f, phic);
        C.coef64 = dalloc<double>(s, (size_t)3 * 8 * C.nmax);
        C.coef32 = dalloc<float>(s, (size_t)3 * 8 * C.nmax);
        launch_coef(s->stream, cx, cy, cz, C.nmax, C.xyz, C.coef64, C.coef32);
        // node types from the coarse level set (it is also passed as g and f, which the
        // classification only checks for finiteness).  Its flags are not read: the coarse
        // level set is a subset of the validated one, and a wall node in a body next to a
        // fluid node is no error on a coarse level (a zero Dirichlet node of the correction)
        C.type = dalloc<int8_t>(s, C.nn);
        launch_classify(s->stream, cx, cy, cz, phic, phic, phic, C.type, cflag);
        launch_mark_irregular(s->stream, cx, cy, cz, C.type);
        int *lst = dalloc<int>(s, C.nn);
        temps.push_back(lst);
        long long cnt;
        count_nodes(s, C.nn, C.type, 2, lst, &cnt);
        C.nirr = (int)cnt;
        C.irr_node = dalloc<int>(s, C.nirr);
        if (C.nirr) ck(hipMemcpyAsync(C.irr_node, lst, C.nirr * sizeof(int), hipMemcpyDeviceToDevice, s->stream));
        C.k64 = dalloc<double>(s, (size_t)7 * C.nirr);
        C.k32 = dalloc<float>(s, (size_t)7 * C.nirr);
        launch_krows(s->stream, cx, cy, cz, C.xyz, C.xyz + cx, C.xyz + cx + cy, phic, C.type, C.nirr, C.irr_node, C.k64);
        launch_to_float(s->stream, (size_t)7 * C.nirr, C.k64, C.k32);
        C.irr_map = dalloc<int>(s, C.nn);
        launch_mg_irr_map(s->stream, C.nirr, C.irr_node, C.irr_map);
        C.skip = dalloc<uint32_t>(s, (size_t)C.g.W * cy * cz + 2);
        launch_fill<uint32_t>(s->stream, (size_t)C.g.W * cy * cz + 2, C.skip, 0u);
        launch_skipbits(s->stream, C.g, C.type, C.skip);
        s->mg.push_back(C);
        hx = hc;
        phi_f = phic;
    }
    sync(s);
    for (void *p : temps) dfree(s, p);
    const int nmax = std::max(s->opt.mg_nu, s->opt.mg_coarse_steps);
    s->mg_c1.assign(nmax, 0.0);
    s->mg_c2.assign(nmax, 0.0);
    s->mg_cc1.assign(nmax, 0.0);
    s->mg_cc2.assign(nmax, 0.0);
    cheb_coefficients(nmax, s->opt.mg_smooth_lo, s->opt.lam_hi, s->mg_c1.data(), s->mg_c2.data());
    const MgLevel &Lc = s->mg.back();
    const double pi = 3.14159265358979323846;
    double lam1 = 0.0;
    for (int d = 0; d < 3; ++d) lam1 += 1.0 - std::cos(pi / (Lc.n[d] - 1));
    lam1 /= 3.0;
    cheb_coefficients(nmax, lam1, s->opt.lam_hi, s->mg_cc1.data(), s->mg_cc2.data());
    // a coarsest level below the problem's grid that fits one workgroup is solved there
    MgLevel &Lc2 = s->mg.back();
    if (s->mg.size() > 1 && (size_t)(Lc2.n[0] - 2) * (Lc2.n[1] - 2) * (Lc2.n[2] - 2) <= (size_t)MG_LDS_NODES) {
        Lc2.lds = true;
        std::vector<double> cc(s->mg_cc1);
        cc.insert(cc.end(), s->mg_cc2.begin(), s->mg_cc2.end());
        std::vector<float> cc32(cc.begin(), cc.end());
        s->mg_ccd64 = upload(s, cc, keep);
        s->mg_ccd32 = upload(s, cc32, keep);
        sync(s);
    }
}

template <typename T>
void precond_standalone(cps_solver *s, const double *rho_dev, double *out_dev)
{
    Vecs<T> V;
    T *all[5];
    for (auto &p : all) {
        p = dalloc<T>(s, s->nn + VEC_PAD);
        launch_fill<T>(s->stream, s->nn + VEC_PAD, p, T(0));
    }
    V.c[0] = all[0]; V.c[1] = all[1];
    T *rin = all[2], *ps = all[3], *dst = all[4];
    launch_masked_copy<double, T>(s->stream, s->nn, s->type, rho_dev, rin);
    // state: alpha = 0 so that the fused first step computes x1 from rho itself
    DevState zero{};
    ck(hipMemcpyAsync(s->st, &zero, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    sync(s);
    double c1[MAX_INNER], c2[MAX_INNER];
    cheb_coefficients(s->opt.inner_iters, s->opt.lam_lo, s->opt.lam_hi, c1, c2);
    precond_apply<T>(s, V, FIRST_S, rin, ps, rin, dst, c1, c2, s->st);
    launch_masked_copy<T, double>(s->stream, s->nn, s->type, dst, out_dev);
    sync(s);
    for (auto p : all) dfree(s, p);
}

}  // namespace

// accessor used by the network's restriction (net.hip)
int cps_internal_fields(cps_solver *s, const double **phi, const double **g, const double **f, int *nx, int *ny, int *nz,
                        void **stream)
{
    *phi = s->phi;
    *g = s->gf;
    *f = s->f;
    *nx = s->nx;
    *ny = s->ny;
    *nz = s->nz;
    *stream = (void *)s->stream;
    return 0;
}

// =========================================================================================
// C-ABI
// =========================================================================================
extern "C" {

void cps_default_options(cps_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(cps_options);
    o->precision = CPS_FP64;
    o->inner_iters = DEFAULT_INNER;
    o->max_iters = 20000;
    o->max_refine = 40;
    o->max_restarts = 5;
    o->device_ptrs = 0;
    o->kernel_timing = 0;
    o->inner_tol = 1e-4;
    o->lam_lo = 0.0;
    o->lam_hi = DEFAULT_LAM_HI;
    o->stream = nullptr;
    o->precond = CPS_PRECOND_MULTIGRID;
    o->mg_levels = MG_MAX_LEVELS;
    o->mg_nu = 2;
    o->mg_coarse_steps = 8;
    o->mg_smooth_lo = 0.2;
    o->sip_iters = 8;
    o->fp64_finish = 1;
    o->sip_alpha = 0.9;
}

const char *cps_strerror(int code)
{
    switch (code) {
    case CPS_OK: return "ok";
    case CPS_EINVAL: return "invalid argument (sizes, coordinates, NaN/Inf input or options)";
    case CPS_EGEOM: return "invalid geometry (a fluid node next to a wall node inside a body, or a singular modified line)";
    case CPS_ENOMEM: return "out of memory";
    case CPS_EDEVICE: return "HIP runtime error or no GPU";
    case CPS_EBREAKDOWN: return "BiCGSTAB breakdown beyond max_restarts";
    case CPS_ENOCONV: return "not converged within max_iters";
    case CPS_ENAN: return "NaN/Inf in the iteration";
    default: return "unknown error";
    }
}

int cps_setup(cps_solver **out, int32_t nx, int32_t ny, int32_t nz, const double *x, const double *y, const double *z,
              const double *phi, const double *g, const double *f, const cps_options *opt)
{
    if (!out || !x || !y || !z || !phi || !g || !f) return CPS_EINVAL;
    *out = nullptr;
    cps_options o;
    cps_default_options(&o);
    if (opt) {
        if (opt->struct_size != (int32_t)sizeof(cps_options)) return CPS_EINVAL;
        o = *opt;
    }
    if (nx < 3 || ny < 3 || nz < 3) return CPS_EINVAL;
    if ((double)nx * ny * nz >= 2147483647.0) return CPS_EINVAL;
    if (o.precision != CPS_FP64 && o.precision != CPS_MIXED) return CPS_EINVAL;
    if (o.inner_iters < 1 || o.inner_iters > MAX_INNER || o.max_iters < 1 || o.max_refine < 1 || o.max_restarts < 0)
        return CPS_EINVAL;
    if (!(o.lam_lo >= 0.0) || !(o.lam_hi > 0.0) || !(o.inner_tol > 0.0 && o.inner_tol < 1.0)) return CPS_EINVAL;
    if (o.lam_lo == 0.0) {
        const double pi = 3.14159265358979323846;
        double lam1 = ((1.0 - std::cos(pi / (nx - 1))) + (1.0 - std::cos(pi / (ny - 1))) +
                       (1.0 - std::cos(pi / (nz - 1)))) / 3.0;
        o.lam_lo = std::max(o.lam_hi / (4.0 * (double)o.inner_iters * (double)o.inner_iters), lam1);
    }
    if (!(o.lam_hi > o.lam_lo)) return CPS_EINVAL;
    if (o.precond != CPS_PRECOND_CHEBYSHEV && o.precond != CPS_PRECOND_MULTIGRID && o.precond != CPS_PRECOND_SIP)
        return CPS_EINVAL;
    if (o.sip_iters < 1 || o.sip_iters > MAX_INNER || !(o.sip_alpha >= 0.0 && o.sip_alpha <= 1.0)) return CPS_EINVAL;
    if (o.fp64_finish != 0 && o.fp64_finish != 1) return CPS_EINVAL;
    if (o.mg_levels < 1 || o.mg_levels > MG_MAX_LEVELS || o.mg_nu < 1 || o.mg_nu > MAX_INNER ||
        o.mg_coarse_steps < 1 || o.mg_coarse_steps > MAX_INNER || !(o.mg_smooth_lo > 0.0) ||
        !(o.mg_smooth_lo < o.lam_hi))
        return CPS_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return CPS_EDEVICE;
    auto t0 = std::chrono::steady_clock::now();
    cps_solver *s = new (std::nothrow) cps_solver();
    if (!s) return CPS_ENOMEM;
    s->opt = o;
    s->stream = (hipStream_t)o.stream;
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->nn = (size_t)nx * ny * nz;
    s->nmax = std::max(nx, std::max(ny, nz));
    s->g = make_geom(nx, ny, nz);
    int rc = CPS_OK;
    try {
        static_assert(2 * sizeof(DevState) <= PINNED_BLOCK / 2, "state copies fit half a pinned block");
        void *blk = pinned_get();
        s->hst = (DevState *)blk;
        s->hscalar = (double *)((char *)blk + PINNED_BLOCK / 2);
        for (auto &e : s->ev) ck(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        // coordinates: validated on the host (they are small)
        std::vector<double> hx(nx + ny + nz);
        const double *srcs[3] = {x, y, z};
        int ns[3] = {nx, ny, nz};
        size_t off = 0;
        s->xyz = dalloc<double>(s, nx + ny + nz);
        for (int d = 0; d < 3; ++d) {
            if (o.device_ptrs) ck(hipMemcpy(hx.data() + off, srcs[d], ns[d] * sizeof(double), hipMemcpyDeviceToHost));
            else std::memcpy(hx.data() + off, srcs[d], ns[d] * sizeof(double));
            for (int q = 0; q < ns[d]; ++q)
                if (!std::isfinite(hx[off + q]) || (q > 0 && !(hx[off + q] > hx[off + q - 1]))) throw CPS_EINVAL;
            off += ns[d];
        }
        ck(hipMemcpyAsync(s->xyz, hx.data(), hx.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
        s->phi = dalloc<double>(s, s->nn);
        s->gf = dalloc<double>(s, s->nn);
        s->f = dalloc<double>(s, s->nn);
        // host fields are uploaded first; device fields are copied by the classification
        // pass itself, which reads them anyway
        if (!o.device_ptrs) {
            to_device(s, s->phi, phi, s->nn * sizeof(double));
            to_device(s, s->gf, g, s->nn * sizeof(double));
            to_device(s, s->f, f, s->nn * sizeof(double));
        }
        // 1D tables
        s->coef64 = dalloc<double>(s, (size_t)3 * 8 * s->nmax);
        s->coef32 = dalloc<float>(s, (size_t)3 * 8 * s->nmax);
        launch_coef(s->stream, nx, ny, nz, s->nmax, s->xyz, s->coef64, s->coef32);
        // classification
        s->type = dalloc<int8_t>(s, s->nn);
        s->dflag = dalloc<int>(s, 1);
        ck(hipMemsetAsync(s->dflag, 0, sizeof(int), s->stream));
        if (o.device_ptrs)
            launch_classify(s->stream, nx, ny, nz, phi, g, f, s->type, s->dflag, s->phi, s->gf, s->f);
        else
            launch_classify(s->stream, nx, ny, nz, s->phi, s->gf, s->f, s->type, s->dflag);
        ck(hipMemcpyAsync(s->hscalar, s->dflag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
        sync(s);
        int flags;
        std::memcpy(&flags, s->hscalar, sizeof(int));
        if (flags & 1) throw CPS_EINVAL;
        if (flags & 2) throw CPS_EGEOM;
        launch_mark_irregular(s->stream, nx, ny, nz, s->type);
        long long cnt;
        s->irr_node = dalloc<int>(s, s->nn);   // trimmed below
        count_type(s, 2, s->irr_node, &cnt);
        s->nirr = (int)cnt;
        {
            // solid and regular counts from one pass over the node types
            int *cnt = dalloc<int>(s, 4);
            ck(hipMemsetAsync(cnt, 0, 4 * sizeof(int), s->stream));
            launch_type_hist(s->stream, s->nn, s->type, cnt);
            int hc[4];
            ck(hipMemcpyAsync(s->hscalar, cnt, sizeof(hc), hipMemcpyDeviceToHost, s->stream));
            sync(s);
            std::memcpy(hc, s->hscalar, sizeof(hc));
            dfree(s, cnt);
            if (hc[2] != s->nirr) throw CPS_EDEVICE;   // the two counts of the irregular nodes disagree
            s->n_solid = hc[3];
            s->n_unknown = (long long)hc[1] + s->nirr;
        }
        {
            int *trimmed = dalloc<int>(s, s->nirr);
            if (s->nirr) ck(hipMemcpyAsync(trimmed, s->irr_node, s->nirr * sizeof(int), hipMemcpyDeviceToDevice, s->stream));
            sync(s);
            dfree(s, s->irr_node);
            s->irr_node = trimmed;
        }
        // two words of zero padding: vectorised kernels read skip words in pairs
        s->skip = dalloc<uint32_t>(s, (size_t)s->g.W * ny * nz + 2);
        launch_fill<uint32_t>(s->stream, (size_t)s->g.W * ny * nz + 2, s->skip, 0u);
        launch_skipbits(s->stream, s->g, s->type, s->skip);
        s->irr_bits = dalloc<uint32_t>(s, (size_t)s->g.W * ny * nz);
        s->irr_wstart = dalloc<int>(s, (size_t)s->g.W * ny * nz);
        launch_irr_words(s->stream, s->g, s->type, s->irr_node, s->nirr, s->irr_bits, s->irr_wstart);
        // reduction scratch: enough for the largest launch
        size_t maxblk = (size_t)std::max({s->g.ta.nblk, s->g.tr.nblk, s->g.tr2.nblk, s->g.tr2s.nblk, s->g.nflat}) +
                        (size_t)(s->nirr + (NT / IRR_LANES) - 1) / (NT / IRR_LANES) + 8;
        s->partials = dalloc<double>(s, 2 * maxblk);
        s->st = dalloc<DevState>(s, 1);
        ck(hipMemsetAsync(s->st, 0, sizeof(DevState), s->stream));
        s->rhs = dalloc<double>(s, s->nn + VEC_PAD);   // read as 4-vectors by the residual
        if (o.precond == CPS_PRECOND_MULTIGRID) {
            // The hierarchy needs the node types and coordinates, not the irregular rows: it
            // is built on a second stream, after the work queued so far, while the rows are
            // built on the solver's stream; its host waits (level sizes) wait for it alone.
            // The rows' host staging is read only after the hierarchy is done.
            ck(hipEventRecord(s->ev[0], s->stream));
            const RowsPending rows = rows_launch(s);
            {
                struct Restore {
                    cps_solver *s;
                    hipStream_t st;
                    ~Restore() { s->stream = st; }
                } restore{s, s->stream};
                const hipStream_t aux = setup_aux_stream();
                ck(hipStreamWaitEvent(aux, s->ev[0], 0));
                s->stream = aux;
                mg_build(s, hx);
            }
            rc = rows_finish(s, rows);
        } else {
            rc = rhs_build(s);
        }
        if (rc == CPS_OK && o.precond == CPS_PRECOND_SIP) sip_build(s);
        sync(s);
    } catch (int code) {
        rc = code;
    } catch (HipFail &) {
        rc = CPS_EDEVICE;
    } catch (std::bad_alloc &) {
        rc = CPS_ENOMEM;
    }
    if (rc != CPS_OK) {
        free_solver(s);
        return rc;
    }
    s->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = s;
    return CPS_OK;
}

int cps_set_rhs(cps_solver *s, const double *f, const double *g)
{
    if (!s || !f || !g) return CPS_EINVAL;
    try {
        to_device(s, s->f, f, s->nn * sizeof(double));
        to_device(s, s->gf, g, s->nn * sizeof(double));
        ck(hipMemsetAsync(s->dflag, 0, sizeof(int), s->stream));
        // re-check finiteness with the classification kernel on a scratch type array
        int8_t *tt = dalloc<int8_t>(s, s->nn);
        launch_classify(s->stream, s->nx, s->ny, s->nz, s->phi, s->gf, s->f, tt, s->dflag);
        ck(hipMemcpyAsync(s->hscalar, s->dflag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
        sync(s);
        dfree(s, tt);
        int flags;
        std::memcpy(&flags, s->hscalar, sizeof(int));
        if (flags & 1) return CPS_EINVAL;
        int rc = rhs_build(s);
        sync(s);
        return rc;
    } catch (HipFail &) {
        return CPS_EDEVICE;
    } catch (std::bad_alloc &) {
        return CPS_ENOMEM;
    }
}

int cps_solve(cps_solver *s, double tol, double *u, int32_t warm_start, cps_stats *stats)
{
    if (!s || !u || !(tol > 0.0)) return CPS_EINVAL;
    if (stats && stats->struct_size != (int32_t)sizeof(cps_stats) && stats->struct_size != 0) return CPS_EINVAL;
    auto t0 = std::chrono::steady_clock::now();
    int status = CPS_ENOCONV;
    int iters = 0, iters32 = 0, refine = 0, restarts = 0;
    double warm_alpha = 0.0;
    DevState ds{};
    try {
        s->tev_used = 0;
        s->sweep_count = 0;
        s->iter_enq = 0;
        s->hist_iter.clear();
        s->hist_true.clear();
        const int m = s->opt.inner_iters;
        double c1[MAX_INNER], c2[MAX_INNER];
        cheb_coefficients(m, s->opt.lam_lo, s->opt.lam_hi, c1, c2);
        const Launch L = s->launch();
        const double tol2 = tol * tol;
        // FP64 solution vector (unknown entries only); the FP64 Krylov set only in FP64 mode
        if (s->opt.precision == CPS_FP64) alloc_vecs<double>(s, s->v64);   // x64 is its x
        if (s->opt.precond == CPS_PRECOND_MULTIGRID) {
            if (s->opt.precision == CPS_FP64) mg_alloc<double>(s); else mg_alloc<float>(s);
        }
        if (!s->x64) s->x64 = dalloc<double>(s, s->nn + VEC_PAD);
        double *x64 = (s->opt.precision == CPS_FP64) ? s->v64.x : s->x64;
        if (warm_start) {
            // a device array is read in place; a host one is staged first
            const double *u_dev = u;
            if (!s->opt.device_ptrs) {
                if (!s->tmp64) s->tmp64 = dalloc<double>(s, s->nn);
                to_device(s, s->tmp64, u, s->nn * sizeof(double));
                u_dev = s->tmp64;
            }
            launch_masked_copy<double, double>(s->stream, s->nn, s->type, u_dev, x64);
            ck(hipMemsetAsync(s->dflag, 0, sizeof(int), s->stream));
            launch_check_finite(s->stream, s->nn, s->type, x64, s->dflag);
            ck(hipMemcpyAsync(s->hscalar, s->dflag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
            sync(s);
            int bad;
            std::memcpy(&bad, s->hscalar, sizeof(int));
            if (bad) launch_fill<double>(s->stream, s->nn, x64, 0.0);   // reject a NaN/Inf warm start
            else warm_alpha = scale_warm_start(s, x64);
        } else {
            launch_fill<double>(s->stream, s->nn, x64, 0.0);
        }
        auto converged = [&](const DevState &d) { return d.res2 <= tol2 * s->bn2 && d.res2s <= tol2 * s->bs2; };
        // Target for the recursive Jacobi-weighted norm: tol^2 ||D^-1 b||^2, tightened in
        // proportion when the paper-scaled norm is the one still above its target.
        auto jacobi_target = [&](const DevState &d) {
            double t2 = tol2 * s->bs2;
            if (d.res2 > tol2 * s->bn2 && d.res2 > 0.0) t2 = std::min(t2, d.res2s * (tol2 * s->bn2 / d.res2));
            return t2;
        };
        // FP64 BiCGSTAB from the current x64 until the true residual converges; a new pass
        // restarts from the true residual after a breakdown or when the recursive residual
        // reached its target but the true one did not
        auto fp64_passes = [&]() -> int {
            alloc_vecs<double>(s, s->v64);
            if (s->opt.precond == CPS_PRECOND_MULTIGRID) mg_alloc<double>(s);
            Vecs<double> &V = s->v64;
            for (int pass = 0, r64 = 0;; ++pass) {
                launch_apply<double, double>(MODE_RES, L, s->cf64(), s->ir64(), x64, V.r, nullptr, s->rhs, s->st);
                ds = read_state(s);
                note_true(s, ds);
                if (!(ds.res2 == ds.res2) || !(ds.res2s == ds.res2s)) return CPS_ENAN;
                if (converged(ds)) return CPS_OK;
                if (iters >= s->opt.max_iters) return CPS_ENOCONV;
                if (pass > 0) {
                    ++restarts;
                    if (++r64 > s->opt.max_restarts) return CPS_EBREAKDOWN;
                }
                const double target2 = jacobi_target(ds);
                set_stop2(s, target2);
                launch_restart<double>(L, s->ir64(), V.r, V.r0, V.p, V.v, s->st);
                // the restart is done at once exactly when the residual already meets the
                // target (it compares the same two values on the device); otherwise the first
                // state read of the run reports a non-finite restart
                DevState d1 = ds;
                if (ds.res2s <= target2) d1.done = 1;
                else d1 = run_iterations<double, double>(s, V, x64, s->opt.max_iters - iters, c1, c2, ds.iters);
                iters += d1.iters - ds.iters;
                if (d1.done == 3) return CPS_ENAN;
            }
        };
        if (s->opt.precision == CPS_FP64) {
            status = fp64_passes();
        } else {
            alloc_vecs<float>(s, s->v32);
            Vecs<float> &V = s->v32;
            double prev2 = -1.0;     // ||D^-1 r||^2 before the last refinement step
            bool finish64 = false;
            for (refine = 0;; ++refine) {
                launch_apply<double, float>(MODE_RES, L, s->cf64(), s->ir64(), x64, V.r, nullptr, s->rhs, s->st);
                ds = read_state(s);
                note_true(s, ds);
                if (!(ds.res2 == ds.res2) || !(ds.res2s == ds.res2s)) { status = CPS_ENAN; break; }
                if (converged(ds)) { status = CPS_OK; break; }
                if (iters >= s->opt.max_iters) { status = CPS_ENOCONV; break; }
                // Every step asks its FP32 solve for at least a 4x reduction of ||D^-1 r||^2;
                // one that reduced it by less than 2x has stagnated (FP32 cannot resolve the
                // correction).  Then, or when the step or restart budget is spent, the solve
                // continues in FP64 (fp64_finish) or stops.
                const bool stalled = prev2 >= 0.0 && !(ds.res2s <= 0.5 * prev2);
                if (stalled || refine >= s->opt.max_refine || restarts > s->opt.max_restarts) {
                    if (s->opt.fp64_finish) {
                        finish64 = true;
                    } else {
                        status = (restarts > s->opt.max_restarts) ? CPS_EBREAKDOWN : CPS_ENOCONV;
                    }
                    break;
                }
                prev2 = ds.res2s;
                // each FP32 solve reduces the residual by inner_tol, the last one just enough
                double target2 = std::max(s->opt.inner_tol * s->opt.inner_tol * ds.res2s, 0.25 * jacobi_target(ds));
                set_stop2(s, target2);
                launch_fill<float>(s->stream, s->nn, V.x, 0.0f);
                launch_restart<float>(L, s->ir32(), V.r, V.r0, V.p, V.v, s->st);
                // done at once exactly when the residual already meets the target (see above)
                DevState d1 = ds;
                if (ds.res2s <= target2) d1.done = 1;
                else d1 = run_iterations<float, float>(s, V, V.x, s->opt.max_iters - iters, c1, c2, ds.iters);
                iters += d1.iters - ds.iters;
                iters32 += d1.iters - ds.iters;
                if (d1.done == 3) { ++restarts; continue; }   // discard a non-finite correction
                if (d1.done == 2) ++restarts;
                launch_add_correction(s->stream, s->nn, x64, V.x);
            }
            if (finish64) {
                s->hist_true.resize(s->hist_true.size() - 2);   // the first FP64 pass recomputes it
                status = fp64_passes();
            }
        }
        // output: unknowns, g on the walls, 0 in the bodies (into a device array directly)
        if (s->opt.device_ptrs) {
            launch_output(s->stream, s->nn, s->type, x64, s->gf, u);
        } else {
            if (!s->tmp64) s->tmp64 = dalloc<double>(s, s->nn);
            launch_output(s->stream, s->nn, s->type, x64, s->gf, s->tmp64);
            from_device(s, u, s->tmp64, s->nn * sizeof(double));
        }
        sync(s);
    } catch (HipFail &) {
        return CPS_EDEVICE;
    } catch (std::bad_alloc &) {
        return CPS_ENOMEM;
    }
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(s, stats, ds, iters, iters32, refine, restarts, status, ms);
    if (stats) stats->warm_alpha = warm_alpha;
    return status;
}

int cps_residual(cps_solver *s, const double *u, double *r, double *rel)
{
    if (!s || !u) return CPS_EINVAL;
    try {
        if (!s->tmp64) s->tmp64 = dalloc<double>(s, s->nn);
        double *xin = dalloc<double>(s, s->nn + VEC_PAD);
        double *rout = dalloc<double>(s, s->nn);
        to_device(s, s->tmp64, u, s->nn * sizeof(double));
        launch_masked_copy<double, double>(s->stream, s->nn, s->type, s->tmp64, xin);
        launch_fill<double>(s->stream, s->nn, rout, 0.0);
        launch_apply<double, double>(MODE_RES, s->launch(), s->cf64(), s->ir64(), xin, rout, nullptr, s->rhs, s->st);
        if (r) from_device(s, r, rout, s->nn * sizeof(double));
        DevState ds = read_state(s);
        if (rel) {
            rel[0] = std::sqrt(ds.res2 / (s->bn2 > 0 ? s->bn2 : 1.0));
            rel[1] = std::sqrt(ds.res2s / (s->bs2 > 0 ? s->bs2 : 1.0));
        }
        dfree(s, xin);
        dfree(s, rout);
    } catch (HipFail &) {
        return CPS_EDEVICE;
    } catch (std::bad_alloc &) {
        return CPS_ENOMEM;
    }
    return CPS_OK;
}

int cps_apply(cps_solver *s, const double *x, double *y, int32_t precision)
{
    if (!s || !x || !y || (precision != CPS_FP64 && precision != CPS_MIXED)) return CPS_EINVAL;
    try {
        if (!s->tmp64) s->tmp64 = dalloc<double>(s, s->nn);
        to_device(s, s->tmp64, x, s->nn * sizeof(double));
        if (precision == CPS_FP64) {
            double *xin = dalloc<double>(s, s->nn + VEC_PAD), *yo = dalloc<double>(s, s->nn);
            launch_masked_copy<double, double>(s->stream, s->nn, s->type, s->tmp64, xin);
            launch_fill<double>(s->stream, s->nn, yo, 0.0);
            launch_apply<double, double>(MODE_PLAIN, s->launch(), s->cf64(), s->ir64(), xin, yo, nullptr, nullptr, nullptr);
            from_device(s, y, yo, s->nn * sizeof(double));
            sync(s);
            dfree(s, xin);
            dfree(s, yo);
        } else {
            float *xin = dalloc<float>(s, s->nn + VEC_PAD), *yo = dalloc<float>(s, s->nn);
            launch_masked_copy<double, float>(s->stream, s->nn, s->type, s->tmp64, xin);
            launch_fill<float>(s->stream, s->nn, yo, 0.0f);
            launch_apply<float, float>(MODE_PLAIN, s->launch(), s->cf32(), s->ir32(), xin, yo, nullptr, nullptr, nullptr);
            launch_masked_copy<float, double>(s->stream, s->nn, s->type, yo, s->tmp64);
            from_device(s, y, s->tmp64, s->nn * sizeof(double));
            sync(s);
            dfree(s, xin);
            dfree(s, yo);
        }
    } catch (HipFail &) {
        return CPS_EDEVICE;
    } catch (std::bad_alloc &) {
        return CPS_ENOMEM;
    }
    return CPS_OK;
}

int cps_precond(cps_solver *s, const double *rho, double *phi, int32_t precision)
{
    if (!s || !rho || !phi || (precision != CPS_FP64 && precision != CPS_MIXED)) return CPS_EINVAL;
    try {
        if (!s->tmp64) s->tmp64 = dalloc<double>(s, s->nn);
        double *out = dalloc<double>(s, s->nn);
        to_device(s, s->tmp64, rho, s->nn * sizeof(double));
        const int timing = s->opt.kernel_timing;
        s->opt.kernel_timing = 0;
        if (precision == CPS_FP64) precond_standalone<double>(s, s->tmp64, out);
        else precond_standalone<float>(s, s->tmp64, out);
        s->opt.kernel_timing = timing;
        from_device(s, phi, out, s->nn * sizeof(double));
        sync(s);
        dfree(s, out);
    } catch (HipFail &) {
        return CPS_EDEVICE;
    } catch (std::bad_alloc &) {
        return CPS_ENOMEM;
    }
    return CPS_OK;
}

int cps_get_rhs(cps_solver *s, double *rhs, int8_t *types)
{
    if (!s) return CPS_EINVAL;
    try {
        if (rhs) from_device(s, rhs, s->rhs, s->nn * sizeof(double));
        if (types) from_device(s, types, s->type, s->nn);
        sync(s);
    } catch (HipFail &) {
        return CPS_EDEVICE;
    }
    return CPS_OK;
}

int cps_get_info(cps_solver *s, int64_t out[6])
{
    if (!s || !out) return CPS_EINVAL;
    out[0] = s->n_unknown;
    out[1] = s->nirr;
    out[2] = s->n_solid;
    out[3] = s->nnz;
    out[4] = s->fallback;
    out[5] = (int64_t)s->nn;
    return CPS_OK;
}

int cps_get_irregular(cps_solver *s, int64_t *node, int64_t *ptr, int64_t *col, double *val, double *krow)
{
    if (!s) return CPS_EINVAL;
    try {
        const int n = s->nirr;
        std::vector<int> tmp;
        auto widen = [&](const int *src, size_t cnt, int64_t *dst) {
            tmp.resize(cnt);
            if (cnt) ck(hipMemcpy(tmp.data(), src, cnt * sizeof(int), hipMemcpyDeviceToHost));
            for (size_t q = 0; q < cnt; ++q) dst[q] = tmp[q];
        };
        sync(s);
        if (node) widen(s->irr_node, n, node);
        if (ptr) widen(s->irr_ptr, (size_t)n + 1, ptr);
        if (col) widen(s->irr_col, (size_t)s->nnz, col);
        if (val && s->nnz) ck(hipMemcpy(val, s->irr_val64, s->nnz * sizeof(double), hipMemcpyDeviceToHost));
        if (krow && n) ck(hipMemcpy(krow, s->irr_k64, (size_t)7 * n * sizeof(double), hipMemcpyDeviceToHost));
    } catch (HipFail &) {
        return CPS_EDEVICE;
    }
    return CPS_OK;
}

int cps_get_history(cps_solver *s, double *iter_res, int32_t cap_iter, int32_t *n_iter, double *true_res,
                    int32_t cap_true, int32_t *n_true)
{
    if (!s || cap_iter < 0 || cap_true < 0 || (cap_iter > 0 && !iter_res) || (cap_true > 0 && !true_res))
        return CPS_EINVAL;
    const size_t ni = s->hist_iter.size(), nt = s->hist_true.size() / 2;
    std::copy_n(s->hist_iter.begin(), std::min<size_t>(ni, (size_t)cap_iter), iter_res);
    std::copy_n(s->hist_true.begin(), 2 * std::min<size_t>(nt, (size_t)cap_true), true_res);
    if (n_iter) *n_iter = (int32_t)ni;
    if (n_true) *n_true = (int32_t)nt;
    return CPS_OK;
}

void cps_destroy(cps_solver *s) { free_solver(s); }

}  // extern "C"
