// setup.hip -- construction of the discrete problem on the GPU, all in FP64:
// 1D compact and second-order coefficients (Eqs. app_xxx, 2ndorder_coef), node
// classification (Sec. 2, Fig. grid_point_types), the ordered list of irregular nodes, the
// modified rows of B at those nodes (Secs. 2.2-2.3), their Shortley-Weller K rows (Sec. 3.3)
// and the right-hand side q + b (Eqs. q, bc, cor).
//
// Readings of the paper used here:
//  * An IBI exists on a grid segment whose end nodes have level sets of opposite sign
//    (phi > 0 fluid, phi <= 0 solid).  Its position is the root, inside the segment, of the
//    degree-5 polynomial interpolating nodal phi at six nodes around the segment (the window
//    is shifted to stay inside the grid); g at the IBI is that interpolation of nodal g.
//  * A modified line window (three nodes along one direction, Eq. lhsrhs_xxyyzz_mod) keeps
//    the row's L weights at its fluid nodes (they form Q-bar) and replaces its R part by a
//    one-sided operator per fluid run whose weights reproduce sum_p L[p] u''(x_p) exactly for
//    all polynomials of degree < |P| -- the Taylor systems of Eqs. mat1-mat4 written as
//    moment conditions.  |P| = 6 (run + extra nodes marching away from the interface + IBI)
//    for a window with one run, 5 per side of an F-S-F window (Sec. 2.3), 3 for S-F-S.  A
//    march that meets a wall node keeps it (known value) and stops; one that meets a solid
//    node ends at that IBI.  Every shortened set is counted as a fallback.
#include <math.h>

#include "cps_device.h"
#include "cps_kernels.h"

namespace cps {

// ---------------------------------------------------------------------------------------
// 1D coefficient tables
// ---------------------------------------------------------------------------------------
// The tables of all three axes in one launch: axis d = blockIdx.y, 8 values per index in FP64
// and FP32; indices n_d .. nmax - 1 of a shorter axis are zero.
__global__ void k_coef(int nx, int ny, int nz, int nmax, const double *__restrict__ xyz, double *__restrict__ coef,
                       float *__restrict__ coef32)
{
    const int d = (int)blockIdx.y;
    const int n = d == 0 ? nx : (d == 1 ? ny : nz);
    const double *t = xyz + (d == 0 ? 0 : (d == 1 ? nx : nx + ny));
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nmax) return;
    double o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i == 0 || i == n - 1) {
        // wall indices: never used by a row; nonzero diagonals keep flat pointwise
        // kernels finite on the (zero) wall entries
        o[3] = -1.0;
        o[6] = -1.0;
    } else if (i < n) {
        double hf = t[i + 1] - t[i], hb = t[i] - t[i - 1];
        // Eq. (app_xxx): denominator (hf + hb)(hf^2 + 3 hf hb + hb^2)
        double den = hf * hf * hf + 4.0 * hf * hf * hb + 4.0 * hf * hb * hb + hb * hb * hb;
        o[0] = hf * (hb * hb + hb * hf - hf * hf) / den;        // a
        o[1] = hb * (hf * hf + hb * hf - hb * hb) / den;        // c
        o[2] = 12.0 * hf / den;                                 // ar
        o[3] = -12.0 / (hf * hf + 3.0 * hf * hb + hb * hb);     // br
        o[4] = 12.0 * hb / den;                                 // cr
        // Eq. (2ndorder_coef)
        o[5] = 2.0 / (hb * (hf + hb));
        o[6] = -2.0 / (hb * hf);
        o[7] = 2.0 / (hf * (hf + hb));
    }
    const size_t at = 8 * ((size_t)d * nmax + i);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        coef[at + q] = o[q];
        coef32[at + q] = (float)o[q];
    }
}

void launch_coef(hipStream_t s, int nx, int ny, int nz, int nmax, const double *xyz, double *coef, float *coef32)
{
    k_coef<<<dim3((unsigned)((nmax + 255) / 256), 3), 256, 0, s>>>(nx, ny, nz, nmax, xyz, coef, coef32);
}

// ---------------------------------------------------------------------------------------
// classification
// ---------------------------------------------------------------------------------------
// one thread per node: x from the thread index, y and z from the grid (no 64-bit divisions);
// with phi_out (then also g_out, f_out) the three fields are copied on the way
__global__ void __launch_bounds__(256) k_classify(int nx, int ny, int nz, const double *__restrict__ phi,
                                                  const double *__restrict__ g, const double *__restrict__ f,
                                                  int8_t *__restrict__ type, int *flags, double *__restrict__ phi_out,
                                                  double *__restrict__ g_out, double *__restrict__ f_out)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int j = (int)(blockIdx.y * blockDim.y + threadIdx.y);
    const int k = (int)blockIdx.z;
    if (i >= nx || j >= ny) return;
    const size_t e = (size_t)i + (size_t)nx * j + (size_t)nx * ny * k;
    const double p = phi[e], gv = g[e], fv = f[e];
    if (!isfinite(p) || !isfinite(gv) || !isfinite(fv)) atomicOr(flags, 1);
    if (phi_out) {
        phi_out[e] = p;
        g_out[e] = gv;
        f_out[e] = fv;
    }
    const bool wall = i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1;
    if (wall) {
        // A wall node may lie in a body (an interior problem) as long as no fluid node is
        // among its interior neighbours, so that no row of the scheme reaches it.
        if (!(p > 0.0)) {
            bool fluid_nb = false;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int a = i + dx, b = j + dy, c = k + dz;
                        if (a < 1 || b < 1 || c < 1 || a > nx - 2 || b > ny - 2 || c > nz - 2) continue;
                        if (phi[(size_t)a + (size_t)nx * b + (size_t)nx * ny * c] > 0.0) fluid_nb = true;
                    }
            if (fluid_nb) atomicOr(flags, 2);
        }
        type[e] = 0;
    } else {
        type[e] = (p > 0.0) ? 1 : 3;
    }
}

void launch_classify(hipStream_t s, int nx, int ny, int nz, const double *phi, const double *g, const double *f,
                     int8_t *type, int *flags, double *phi_out, double *g_out, double *f_out)
{
    dim3 blk(64, 4), grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4), (unsigned)nz);
    k_classify<<<grid, blk, 0, s>>>(nx, ny, nz, phi, g, f, type, flags, phi_out, g_out, f_out);
}

// a fluid node with a solid node among its 26 neighbours is irregular (one thread per
// interior node; a neighbour read while it turns from regular to irregular is never solid)
__global__ void __launch_bounds__(256) k_mark_irregular(int nx, int ny, int nz, int8_t *__restrict__ type)
{
    const int i = 1 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int j = 1 + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    const int k = 1 + (int)blockIdx.z;
    if (i > nx - 2 || j > ny - 2) return;
    const size_t plane = (size_t)nx * ny;
    const size_t e = (size_t)i + (size_t)nx * j + plane * k;
    if (type[e] != 1) return;
    bool irr = false;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                irr |= type[e + dx + (ptrdiff_t)dy * nx + (ptrdiff_t)dz * (ptrdiff_t)plane] == 3;
    if (irr) type[e] = 2;
}

void launch_mark_irregular(hipStream_t s, int nx, int ny, int nz, int8_t *type)
{
    if (nx < 3 || ny < 3 || nz < 3) return;
    dim3 blk(64, 4), grid((unsigned)((nx - 2 + 63) / 64), (unsigned)((ny - 2 + 3) / 4), (unsigned)(nz - 2));
    k_mark_irregular<<<grid, blk, 0, s>>>(nx, ny, nz, type);
}

// ---------------------------------------------------------------------------------------
// ordered stream compaction (counts per block -> scan -> scatter)
// ---------------------------------------------------------------------------------------
constexpr int CMP_THREADS = 256, CMP_PER_THREAD = 32, CMP_CHUNK = CMP_THREADS * CMP_PER_THREAD;

// the CMP_PER_THREAD node types of one thread (from 16-byte loads where the chunk is whole)
__device__ __forceinline__ void load_types(size_t n, const int8_t *__restrict__ type, size_t base,
                                           int8_t (&t)[CMP_PER_THREAD])
{
    if (base + CMP_PER_THREAD <= n) {
#pragma unroll
        for (int h = 0; h < CMP_PER_THREAD / 16; ++h) {
            const int4 v = *reinterpret_cast<const int4 *>(type + base + 16 * h);
            const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int u = 0; u < 16; ++u) t[16 * h + u] = (int8_t)((w[u >> 2] >> (8 * (u & 3))) & 0xff);
        }
    } else {
#pragma unroll
        for (int q = 0; q < CMP_PER_THREAD; ++q) t[q] = base + q < n ? type[base + q] : (int8_t)-1;
    }
}

int compact_blocks(size_t n) { return (int)((n + CMP_CHUNK - 1) / CMP_CHUNK); }

__global__ void k_count(size_t n, const int8_t *__restrict__ type, int8_t want, int *blockcnt)
{
    __shared__ int sh[CMP_THREADS];
    size_t base = (size_t)blockIdx.x * CMP_CHUNK + (size_t)threadIdx.x * CMP_PER_THREAD;
    int8_t t[CMP_PER_THREAD];
    load_types(n, type, base, t);
    int c = 0;
#pragma unroll
    for (int q = 0; q < CMP_PER_THREAD; ++q) c += t[q] == want;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int o = CMP_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = sh[0];
}

__global__ void k_scatter(size_t n, const int8_t *__restrict__ type, int8_t want, const int *__restrict__ offs,
                          int *__restrict__ list)
{
    __shared__ int sh[CMP_THREADS];
    size_t base = (size_t)blockIdx.x * CMP_CHUNK + (size_t)threadIdx.x * CMP_PER_THREAD;
    int8_t t[CMP_PER_THREAD];
    load_types(n, type, base, t);
    int c = 0;
#pragma unroll
    for (int q = 0; q < CMP_PER_THREAD; ++q) c += t[q] == want;
    sh[threadIdx.x] = c;
    __syncthreads();
    // inclusive scan (Hillis-Steele) over the block
    for (int o = 1; o < CMP_THREADS; o <<= 1) {
        int v = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int pos = offs[blockIdx.x] + sh[threadIdx.x] - c;
#pragma unroll
    for (int q = 0; q < CMP_PER_THREAD; ++q)
        if (t[q] == want) list[pos++] = (int)(base + q);
}

// exclusive scan of n ints by one block; out[n] = total.  Each round covers SCAN_PT
// consecutive elements per thread: a thread sums its run, the block scans the 1024 run sums
// (Hillis-Steele in LDS), and each thread writes its run's prefixes.
constexpr int SCAN_PT = 16;
__global__ void __launch_bounds__(1024) k_scan(const int *__restrict__ in, int *__restrict__ out, int n)
{
    __shared__ int sh[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024 * SCAN_PT) {
        const int b0 = base + (int)threadIdx.x * SCAN_PT;
        int v[SCAN_PT], sum = 0;
#pragma unroll
        for (int u = 0; u < SCAN_PT; ++u) {
            v[u] = b0 + u < n ? in[b0 + u] : 0;
            sum += v[u];
        }
        sh[threadIdx.x] = sum;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int a = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        int run = carry + sh[threadIdx.x] - sum;
#pragma unroll
        for (int u = 0; u < SCAN_PT; ++u) {
            if (b0 + u < n) out[b0 + u] = run;
            run += v[u];
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

void launch_scan(hipStream_t s, const int *in, int *out, int n) { k_scan<<<1, 1024, 0, s>>>(in, out, n); }

__global__ void k_copy_count(const int *__restrict__ src, int *__restrict__ dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

void launch_compact(hipStream_t s, size_t n, const int8_t *type, int8_t want, int *blockcnt, int *list, int *count,
                    int nblocks)
{
    // blockcnt holds 2*nblocks+1 ints: counts, then the exclusive offsets (+ total)
    k_count<<<nblocks, CMP_THREADS, 0, s>>>(n, type, want, blockcnt);
    k_scan<<<1, 1024, 0, s>>>(blockcnt, blockcnt + nblocks, nblocks);
    k_scatter<<<nblocks, CMP_THREADS, 0, s>>>(n, type, want, blockcnt + nblocks, list);
    k_copy_count<<<1, 64, 0, s>>>(blockcnt + 2 * nblocks, count);   // the total, on the device
}

// skip bits: solid or irregular interior nodes
__global__ void k_skipbits(Geom g, const int8_t *__restrict__ type, uint32_t *__restrict__ skip)
{
    size_t nw = (size_t)g.W * g.ny * g.nz;
    for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (size_t)gridDim.x * blockDim.x) {
        size_t line = w / g.W;
        int i0 = (int)(w % g.W) * 32;
        uint32_t bits = 0;
        for (int q = 0; q < 32; ++q) {
            int i = i0 + q;
            if (i >= g.nx) break;
            int8_t t = type[line * g.nx + i];
            if (t == 2 || t == 3) bits |= 1u << q;
        }
        skip[w] = bits;
    }
}

void launch_skipbits(hipStream_t s, const Geom &g, const int8_t *type, uint32_t *skip)
{
    size_t nw = (size_t)g.W * g.ny * g.nz;
    k_skipbits<<<(unsigned)std::min<size_t>((nw + 255) / 256, 65536), 256, 0, s>>>(g, type, skip);
}

// irregular-node bits per word, and the number of irregular rows (nodes in ascending
// order) before the word's first node: a binary search in the row list
__global__ void k_irr_words(Geom g, const int8_t *__restrict__ type, const int *__restrict__ nodes, int nirr,
                            uint32_t *__restrict__ bits, int *__restrict__ wstart)
{
    size_t nw = (size_t)g.W * g.ny * g.nz;
    for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (size_t)gridDim.x * blockDim.x) {
        size_t line = w / g.W;
        int i0 = (int)(w % g.W) * 32;
        uint32_t b = 0;
        for (int q = 0; q < 32; ++q) {
            int i = i0 + q;
            if (i >= g.nx) break;
            if (type[line * g.nx + i] == 2) b |= 1u << q;
        }
        bits[w] = b;
        const long long first = (long long)line * g.nx + i0;
        int lo = 0, hi = nirr;           // first row whose node is >= first
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if ((long long)nodes[mid] < first) lo = mid + 1;
            else hi = mid;
        }
        wstart[w] = lo;
    }
}

void launch_irr_words(hipStream_t s, const Geom &g, const int8_t *type, const int *nodes, int nirr, uint32_t *bits,
                      int *wstart)
{
    size_t nw = (size_t)g.W * g.ny * g.nz;
    k_irr_words<<<(unsigned)std::min<size_t>((nw + 255) / 256, 65536), 256, 0, s>>>(g, type, nodes, nirr, bits, wstart);
}

// ---------------------------------------------------------------------------------------
// irregular rows
// ---------------------------------------------------------------------------------------
struct Ctx {
    int n[3];
    size_t stride[3];
    const double *t[3];
    const double *coef[3];
    const double *phi, *g, *f;
    const int8_t *type;
    // optional table of the IBIs next to the irregular nodes (null: found where needed):
    // entry 6 row + 2 d + s is the IBI on the segment from the row's node toward its -d
    // (s = 0) or +d (s = 1) neighbour when that neighbour is solid; the row of a node comes
    // from the irregular-node bits (W words per grid row) and the per-word row counts
    const double *ibi_t, *ibi_g;
    const uint32_t *irr_bits;
    const int *irr_wstart;
    int W;
};

constexpr int NSLOT = 27 + 3 * 2 * 4 * 9;   // 3x3x3 box + extra points 2..5 cells out along a line

// slot of a node at offset o from the row node, or -1
__device__ __forceinline__ int slot_of(const int o[3])
{
    int far = -1;
    for (int d = 0; d < 3; ++d)
        if (o[d] < -1 || o[d] > 1) {
            if (far >= 0) return -1;
            far = d;
        }
    if (far < 0) return (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1);
    int m = o[far] < 0 ? -o[far] : o[far];
    if (m > 5) return -1;
    int d1 = (far + 1) % 3, d2 = (far + 2) % 3;
    return 27 + (((far * 2 + (o[far] > 0)) * 4 + (m - 2)) * 9 + (o[d1] + 1) * 3 + (o[d2] + 1));
}

// Interpolating polynomial of degree M-1 through (ts, vs) in Newton form (in place).  The
// point count is a template parameter so that every array index is static and the arrays
// stay in registers (a dynamically indexed private array lives in slow scratch memory).
template <int M>
__device__ __forceinline__ void newton_coeffs(const double (&ts)[M], double (&c)[M])
{
#pragma unroll
    for (int lvl = 1; lvl < M; ++lvl)
#pragma unroll
        for (int q = M - 1; q >= lvl; --q) c[q] = (c[q] - c[q - 1]) / (ts[q] - ts[q - lvl]);
}

template <int M>
__device__ __forceinline__ double newton_eval(const double (&ts)[M], const double (&c)[M], double t, double *deriv)
{
    double p = c[M - 1], dp = 0.0;
#pragma unroll
    for (int q = M - 2; q >= 0; --q) {
        dp = dp * (t - ts[q]) + p;
        p = p * (t - ts[q]) + c[q];
    }
    if (deriv) *deriv = dp;
    return p;
}

// IBI between grid indices `ifl` (fluid) and `isol` (solid) on the line along d through
// node `line0`, from the M-point window starting at index lo.
template <int M>
__device__ __forceinline__ double ibi_window(const Ctx &C, int d, size_t line0, int lo, int ifl, int isol, double *gval,
                                             double *frac)
{
    double ts[M], cp[M], cg[M];
#pragma unroll
    for (int q = 0; q < M; ++q) {
        size_t node = line0 + (size_t)(lo + q) * C.stride[d];
        ts[q] = C.t[d][lo + q];
        cp[q] = C.phi[node];
        cg[q] = C.g[node];
    }
    newton_coeffs<M>(ts, cp);
    newton_coeffs<M>(ts, cg);
    double tf = C.t[d][ifl], tsol = C.t[d][isol];
    double root;
    if (C.phi[line0 + (size_t)isol * C.stride[d]] == 0.0) {
        root = tsol;
    } else {
        // safeguarded Newton: keep the bracket [fluid side (> 0), solid side (<= 0)]
        double a = tf, b = tsol;
        root = 0.5 * (a + b);
        for (int it = 0; it < 200; ++it) {
            double dv, v = newton_eval<M>(ts, cp, root, &dv);
            if (v > 0.0) a = root; else b = root;
            double nxt = (dv != 0.0) ? root - v / dv : 0.5 * (a + b);
            bool inside = (a < b) ? (nxt > a && nxt < b) : (nxt < a && nxt > b);
            if (!inside) nxt = a + 0.5 * (b - a);
            if (nxt == root || nxt == a || nxt == b) { root = nxt; break; }
            root = nxt;
        }
    }
    *gval = newton_eval<M>(ts, cg, root, nullptr);
    *frac = fabs(root - tf) / fabs(tsol - tf);
    return root;
}

// IBI on the segment between node index `ifl` (fluid) and `isol` (solid) of the grid line
// along d through node `line0` (index 0 along d); returns its coordinate, g there, and the
// fraction of the segment between the fluid node and the IBI.  The interpolation window
// holds min(n, 6) nodes around the segment, shifted to stay in the grid.
__device__ double ibi_on_segment(const Ctx &C, int d, size_t line0, int ifl, int isol, double *gval, double *frac)
{
    int n = C.n[d];
    int m = n < 6 ? n : 6;
    int lo = min(ifl, isol) - 2;
    lo = max(0, min(lo, n - m));
    switch (m) {
    case 6: return ibi_window<6>(C, d, line0, lo, ifl, isol, gval, frac);
    case 5: return ibi_window<5>(C, d, line0, lo, ifl, isol, gval, frac);
    case 4: return ibi_window<4>(C, d, line0, lo, ifl, isol, gval, frac);
    default: return ibi_window<3>(C, d, line0, lo, ifl, isol, gval, frac);
    }
}

// The IBI between node index `ifl` (fluid) and its neighbour `isol` (solid) on the line along
// d through the node with coordinates `base` (base[d] ignored; line0 is its index with
// base[d] = 0): read from the table when the fluid node is irregular (always, when the
// neighbour is solid: a fluid node next to a solid one is irregular), else found here.  The
// table holds the values ibi_on_segment returns, so both routes give the same bits.
__device__ double ibi_cached(const Ctx &C, int d, const int base[3], size_t line0, int ifl, int isol, double *gval,
                             double *frac)
{
    if (C.ibi_t) {
        int c[3] = {base[0], base[1], base[2]};
        c[d] = ifl;
        const size_t word = ((size_t)c[2] * C.n[1] + c[1]) * C.W + (c[0] >> 5);
        const uint32_t bits = C.irr_bits[word];
        if ((bits >> (c[0] & 31)) & 1u) {
            const size_t row = (size_t)C.irr_wstart[word] + __popc(bits & ((1u << (c[0] & 31)) - 1u));
            const size_t ent = 6 * row + 2 * d + (isol > ifl ? 1 : 0);
            const double root = C.ibi_t[ent];
            const double tf = C.t[d][ifl], tsol = C.t[d][isol];
            *gval = C.ibi_g[ent];
            *frac = fabs(root - tf) / fabs(tsol - tf);
            return root;
        }
    }
    return ibi_on_segment(C, d, line0, ifl, isol, gval, frac);
}

// The IBI table: one thread per (irregular row, arm); arms toward a neighbour that is not
// solid are left untouched (never read).
__global__ void __launch_bounds__(256) k_ibi_table(Ctx C, int nirr, const int *__restrict__ nodes,
                                                   double *__restrict__ ibi_t, double *__restrict__ ibi_g)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int row = t / 6, arm = t % 6;
    if (row >= nirr) return;
    const int d = arm >> 1, side = arm & 1;
    const size_t rownode = (size_t)nodes[row];
    const int nx = C.n[0], ny = C.n[1];
    const int idx[3] = {(int)(rownode % nx), (int)((rownode / nx) % ny), (int)(rownode / ((size_t)nx * ny))};
    const size_t nb = side ? rownode + C.stride[d] : rownode - C.stride[d];
    if (C.type[nb] != 3) return;
    const size_t line0 = rownode - (size_t)idx[d] * C.stride[d];
    double gv, fr;
    ibi_t[6 * (size_t)row + arm] = ibi_on_segment(C, d, line0, idx[d], side ? idx[d] + 1 : idx[d] - 1, &gv, &fr);
    ibi_g[6 * (size_t)row + arm] = gv;
}

// Solve the NP x NP system A w = rhs by elimination with row pivoting (row swaps by
// selects over static indices, so that A stays in registers).
template <int NP>
__device__ __forceinline__ bool small_solve(double (&A)[NP][NP], double (&rhs)[NP], double (&w)[NP])
{
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        int pr = c;
        double best = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < NP; ++r)
            if (fabs(A[r][c]) > best) { best = fabs(A[r][c]); pr = r; }
        if (best == 0.0) return false;
#pragma unroll
        for (int r = c + 1; r < NP; ++r) {
            const bool sw = r == pr;
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const double tc = A[c][q], tr = A[r][q];
                A[c][q] = sw ? tr : tc;
                A[r][q] = sw ? tc : tr;
            }
            const double bc = rhs[c], br = rhs[r];
            rhs[c] = sw ? br : bc;
            rhs[r] = sw ? bc : br;
        }
#pragma unroll
        for (int r = c + 1; r < NP; ++r) {
            double l = A[r][c] / A[c][c];
#pragma unroll
            for (int q = c; q < NP; ++q) A[r][q] -= l * A[c][q];
            rhs[r] -= l * rhs[c];
        }
    }
#pragma unroll
    for (int r = NP - 1; r >= 0; --r) {
        double acc = rhs[r];
#pragma unroll
        for (int q = r + 1; q < NP; ++q) acc -= A[r][q] * w[q];
        w[r] = acc / A[r][r];
    }
    return true;
}

// Three values picked by a run-time index through selects: a private array indexed at run
// time would live in scratch memory.
struct D3 {
    double v0, v1, v2;
    __device__ __forceinline__ double operator[](int q) const { return q == 0 ? v0 : (q == 1 ? v1 : v2); }
};
__device__ __forceinline__ D3 pick3(int d, const D3 &a, const D3 &b, const D3 &c)
{
    return D3{d == 0 ? a.v0 : (d == 1 ? b.v0 : c.v0), d == 0 ? a.v1 : (d == 1 ? b.v1 : c.v1),
              d == 0 ? a.v2 : (d == 1 ? b.v2 : c.v2)};
}

// One-sided weights on NP points (coordinates pt) that reproduce sum over the run of
// Ld[p] u''(x_p) for every polynomial of degree < NP: the moment conditions in coordinates
// scaled by the reference point tref and the largest offset href.
template <int NP>
__device__ __forceinline__ bool onesided_weights(const double *pt, const double *tr, int plo, int phi_, const D3 Ld,
                                                 double tref, double href, double *wout)
{
    double A[NP][NP], rhs[NP], w[NP];
    double xi[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) xi[q] = (pt[q] - tref) / href;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        double s = 0.0;
        if (m >= 2)
            for (int p = plo; p <= phi_; ++p) {
                double x = (tr[p] - tref) / href;
                double pw = 1.0;
                for (int q = 0; q < m - 2; ++q) pw *= x;
                s += Ld[p + 1] * (double)(m * (m - 1)) * pw;
            }
        rhs[m] = s / (href * href);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            double pw = 1.0;
#pragma unroll
            for (int e = 0; e < m; ++e) pw *= xi[q];
            A[m][q] = pw;
        }
    }
    if (!small_solve<NP>(A, rhs, w)) return false;
#pragma unroll
    for (int q = 0; q < NP; ++q) wout[q] = w[q];
    return true;
}

// The contributions of one window, in the order they are made: (slot, value) for a
// coefficient on an unknown, (-1, value) for a term moved to the right-hand side.  A window
// makes at most 2 runs x 5 points (F-S-F) or 6 points (one run); 12 leaves room.
constexpr int WIN_CAP = 12;
struct WinList {
    double v[WIN_CAP];
    int16_t slot[WIN_CAP];
    int n;
    __device__ __forceinline__ void add(int sl, double c)
    {
        if (n < WIN_CAP) {
            v[n] = c;
            slot[n] = (int16_t)sl;
        }
        ++n;
    }
    __device__ __forceinline__ void rhs_add(double c) { add(-1, c); }
};

// coefficient c on the node at offset o (from the row node): unknown -> slot; wall -> RHS
__device__ __forceinline__ void put(const Ctx &C, WinList &R, size_t rownode, const int o[3], double c)
{
    size_t node = rownode + (ptrdiff_t)o[0] * (ptrdiff_t)C.stride[0] + (ptrdiff_t)o[1] * (ptrdiff_t)C.stride[1] +
                  (ptrdiff_t)o[2] * (ptrdiff_t)C.stride[2];
    int8_t ty = C.type[node];
    if (ty == 0) {
        R.rhs_add(-c * C.g[node]);
        return;
    }
    int sl = slot_of(o);
    if (sl < 0) return;  // unreachable for marches of at most 5 cells
    R.add(sl, c);
}

// Working storage of one lane's one-sided operator: its points (coordinate, offset along
// the line from the window centre, IBI or grid node, g at an IBI) and weights.  It lives
// in LDS: the point list grows in a data-dependent order, and as a private array it would
// sit in scratch memory.
constexpr int PT_CAP = 6;   // one run: <= 2 nodes + IBI + march to 6 points; S-F-S: 3
struct PtBuf {
    double *t, *g, *w;
    signed char *off;
    bool *ibi;
};

// one fluid run [plo, phi_] (positions -1..1 along d of the window centred at `wc` = row
// offset) of a window meeting the body
__device__ __forceinline__ void run_operator(const Ctx &C, WinList &R, size_t rownode, const int rowidx[3], int d, const int wc[3],
                             int plo, int phi_, const bool sol[3], int nruns, const D3 Ld, double W, int &fb,
                             double &minhb, int *bad, PtBuf P)
{
    const int n = C.n[d];
    int cidx = rowidx[d];   // window centre index along d (same as the row's)
    int base[3] = {rowidx[0] + wc[0], rowidx[1] + wc[1], rowidx[2] + wc[2]};
    base[d] = 0;
    size_t line0 = (size_t)base[0] * C.stride[0] + (size_t)base[1] * C.stride[1] + (size_t)base[2] * C.stride[2];
    bool sl = plo > -1 && sol[plo - 1 + 1];
    bool sr = phi_ < 1 && sol[phi_ + 1 + 1];
    int np = 0;
    auto push = [&](double t, int off, bool ibi, double gv) {
        if (np >= PT_CAP) return;
        P.t[np] = t;
        P.off[np] = (signed char)off;
        P.ibi[np] = ibi;
        P.g[np] = gv;
        ++np;
    };
    bool shortened = false;
    double gv, fr;
    if (sl && sr) {
        double tl = ibi_cached(C, d, base, line0, cidx + plo, cidx + plo - 1, &gv, &fr);
        minhb = fmin(minhb, fr);
        push(tl, 0, true, gv);
        for (int p = plo; p <= phi_; ++p) push(C.t[d][cidx + p], p, false, 0.0);
        double th = ibi_cached(C, d, base, line0, cidx + phi_, cidx + phi_ + 1, &gv, &fr);
        minhb = fmin(minhb, fr);
        push(th, 0, true, gv);
        shortened = true;
    } else {
        const int want = (nruns == 2) ? 5 : 6;
        for (int p = plo; p <= phi_; ++p) push(C.t[d][cidx + p], p, false, 0.0);
        int near = sr ? phi_ : plo;                 // run node next to the interface
        int step = sr ? -1 : 1;                     // march away from the interface
        double tb = ibi_cached(C, d, base, line0, cidx + near, cidx + near - step, &gv, &fr);
        minhb = fmin(minhb, fr);
        push(tb, 0, true, gv);
        int pos = sr ? plo : phi_;
        while (np < want) {
            int nxt = pos + step;
            int gi = cidx + nxt;
            if (gi < 0 || gi >= n) { shortened = true; break; }
            size_t node = line0 + (size_t)gi * C.stride[d];
            int8_t ty = C.type[node];
            if (ty == 3) {
                double te = ibi_cached(C, d, base, line0, cidx + pos, gi, &gv, &fr);
                minhb = fmin(minhb, fr);
                push(te, 0, true, gv);
                shortened = true;
                break;
            }
            push(C.t[d][gi], nxt, false, 0.0);
            pos = nxt;
            if (ty == 0) break;   // a wall node: known value, nothing beyond it
        }
        if (np < want) shortened = true;
    }
    if (shortened) ++fb;
    // moment conditions in scaled coordinates
    double tref = C.t[d][cidx + ((sl && sr) ? plo : (sr ? phi_ : plo))];
    double href = 0.0;
    for (int q = 0; q < np; ++q) href = fmax(href, fabs(P.t[q] - tref));
    const double *tr = C.t[d] + cidx;
    bool ok;
    switch (np) {
    case 2: ok = onesided_weights<2>(P.t, tr, plo, phi_, Ld, tref, href, P.w); break;
    case 3: ok = onesided_weights<3>(P.t, tr, plo, phi_, Ld, tref, href, P.w); break;
    case 4: ok = onesided_weights<4>(P.t, tr, plo, phi_, Ld, tref, href, P.w); break;
    case 5: ok = onesided_weights<5>(P.t, tr, plo, phi_, Ld, tref, href, P.w); break;
    case 6: ok = onesided_weights<6>(P.t, tr, plo, phi_, Ld, tref, href, P.w); break;
    default: ok = false;
    }
    if (!ok) {
        atomicOr(bad, 1);   // singular (or impossible) one-sided system: reported to the host
        return;
    }
    for (int q = 0; q < np; ++q) {
        double c = W * P.w[q];
        if (P.ibi[q]) {
            R.rhs_add(-c * P.g[q]);
        } else {
            int o[3] = {wc[0], wc[1], wc[2]};
            o[d] = P.off[q];
            put(C, R, rownode, o, c);
        }
    }
}

// Shortley-Weller K row at the node `rownode` = (idx): Eqs. 2ndorder_coef_mod, A7_mod.  Output
// [diag, -x, +x, -y, +y, -z, +z]; a neighbour that is not an unknown gets 0 (zero Dirichlet
// data), a solid neighbour moves the arm to the interface intersection.
__device__ void sw_krow(const Ctx &C, size_t rownode, const int idx[3], double *out)
{
    double kr[7];
    kr[0] = 0.0;
    for (int d = 0; d < 3; ++d) {
        int b0[3] = {idx[0], idx[1], idx[2]};
        b0[d] = 0;
        size_t line0 = (size_t)b0[0] * C.stride[0] + (size_t)b0[1] * C.stride[1] + (size_t)b0[2] * C.stride[2];
        size_t nm = rownode - C.stride[d], npl = rownode + C.stride[d];
        double hb = C.t[d][idx[d]] - C.t[d][idx[d] - 1], hf = C.t[d][idx[d] + 1] - C.t[d][idx[d]];
        double gv, fr;
        if (C.type[nm] == 3) hb = C.t[d][idx[d]] - ibi_cached(C, d, b0, line0, idx[d], idx[d] - 1, &gv, &fr);
        if (C.type[npl] == 3) hf = ibi_cached(C, d, b0, line0, idx[d], idx[d] + 1, &gv, &fr) - C.t[d][idx[d]];
        kr[0] += -2.0 / (hb * hf);
        int8_t tm = C.type[nm], tp = C.type[npl];
        kr[1 + 2 * d] = (tm == 1 || tm == 2) ? 2.0 / (hb * (hf + hb)) : 0.0;
        kr[2 + 2 * d] = (tp == 1 || tp == 2) ? 2.0 / (hf * (hf + hb)) : 0.0;
    }
    for (int q = 0; q < 7; ++q) out[q] = kr[q];
}

// K rows only (a coarse level of the multigrid preconditioner), the arithmetic of sw_krow
// spread over eight lanes per row: lane 2d + s (s = 0: -d side, 1: +d side; lanes 6, 7 idle)
// finds its arm length (to the neighbour, or to the interface when the neighbour is solid)
// and its off-diagonal entry; lane 0 sums the three diagonal terms in the order d = 0, 1, 2.
__global__ void __launch_bounds__(256) k_krows(Ctx C, int nirr, const int *__restrict__ nodes,
                                               double *__restrict__ k7)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int row = t >> 3, lane = t & 7;
    const bool live = row < nirr && lane < 6;
    const int d = live ? lane >> 1 : 0, side = lane & 1;
    double h = 1.0;
    int8_t tn = 0;
    if (live) {
        const size_t rownode = (size_t)nodes[row];
        const int nx = C.n[0], ny = C.n[1];
        const int idx[3] = {(int)(rownode % nx), (int)((rownode / nx) % ny), (int)(rownode / ((size_t)nx * ny))};
        const int id = d == 0 ? idx[0] : (d == 1 ? idx[1] : idx[2]);
        const size_t sd = d == 0 ? C.stride[0] : (d == 1 ? C.stride[1] : C.stride[2]);
        const double *td = d == 0 ? C.t[0] : (d == 1 ? C.t[1] : C.t[2]);
        const size_t line0 = rownode - (size_t)id * sd;
        const size_t nb = side ? rownode + sd : rownode - sd;
        tn = C.type[nb];
        const int in = side ? id + 1 : id - 1;
        h = side ? td[id + 1] - td[id] : td[id] - td[id - 1];
        if (tn == 3) {
            double gv, fr;
            const double tb = ibi_on_segment(C, d, line0, id, in, &gv, &fr);
            h = side ? tb - td[id] : td[id] - tb;
        }
    }
    const double other = __shfl_xor(h, 1, 8);          // the opposite arm of direction d
    const double hb = side ? other : h, hf = side ? h : other;
    const double diag = -2.0 / (hb * hf);
    const double off = (tn == 1 || tn == 2) ? (side ? 2.0 / (hf * (hf + hb)) : 2.0 / (hb * (hf + hb))) : 0.0;
    const double d1 = __shfl(diag, 2, 8), d2 = __shfl(diag, 4, 8);
    if (!live) return;
    double *out = k7 + 7 * (size_t)row;
    out[1 + lane] = off;
    if (lane == 0) out[0] = ((0.0 + diag) + d1) + d2;
}

// gather of the coarse level set: coarse node (I, J, K) <- fine node (ix[I], iy[J], iz[K])
__global__ void k_gather3(int ncx, int ncy, int ncz, int nfx, int nfy, const int *__restrict__ ix,
                          const int *__restrict__ iy, const int *__restrict__ iz, const double *__restrict__ src,
                          double *__restrict__ dst)
{
    const int I = (int)(blockIdx.x * blockDim.x + threadIdx.x), J = (int)blockIdx.y, K = (int)blockIdx.z;
    if (I >= ncx) return;
    dst[(size_t)I + (size_t)ncx * (J + (size_t)ncy * K)] = src[(size_t)ix[I] + (size_t)nfx * (iy[J] + (size_t)nfy * iz[K])];
}

// One irregular row per 32-lane group (four rows per 128-thread block).  Lanes 0..26 take
// the 27 windows of Eq. lhsrhs_xxyyzz_mod (direction d = lane / 9, cross offsets from
// lane % 9) and list their contributions in LDS; lane 27 forms the row's Q-bar term and its
// Shortley-Weller K row.  The row's lanes then sum the lists in window order into the row's
// slots (a fixed order: reruns are bitwise equal) and emit the row in slot order.
constexpr int BR_ROWS = 4;          // rows per block
constexpr int BR_LANES = 32;        // lanes per row
__global__ void __launch_bounds__(BR_ROWS * BR_LANES) k_build_rows(
    Ctx C, int nirr, const int *__restrict__ nodes, int cap, int *__restrict__ ell_col, double *__restrict__ ell_val,
    int *__restrict__ len, double *__restrict__ rhs_row, double *__restrict__ k7, double *__restrict__ bdiag,
    double *__restrict__ minhb_row, int *__restrict__ fb_row, int *__restrict__ bad)
{
    __shared__ WinList wl[BR_ROWS][27];
    __shared__ double pt_t[BR_ROWS * 27][PT_CAP], pt_g[BR_ROWS * 27][PT_CAP], pt_w[BR_ROWS * 27][PT_CAP];
    __shared__ signed char pt_off[BR_ROWS * 27][PT_CAP];
    __shared__ bool pt_ibi[BR_ROWS * 27][PT_CAP];
    __shared__ double qbar[BR_ROWS];
    __shared__ double slot_sum[BR_ROWS][NSLOT];
    __shared__ int wfb[BR_ROWS][27];
    __shared__ double wminhb[BR_ROWS][27];
    const int grp = threadIdx.x / BR_LANES, lane = threadIdx.x % BR_LANES;
    const int row = blockIdx.x * BR_ROWS + grp;
    const bool live = row < nirr;
    const size_t rownode = live ? (size_t)nodes[row] : 0;
    const int nx = C.n[0], ny = C.n[1];
    const int idx[3] = {(int)(rownode % nx), (int)((rownode / nx) % ny), (int)(rownode / ((size_t)nx * ny))};
    // the row's compact weights along x, y, z: L (left-hand side) and R (second derivative)
    D3 Lx{0, 1, 0}, Ly{0, 1, 0}, Lz{0, 1, 0}, Rx{0, 0, 0}, Ry{0, 0, 0}, Rz{0, 0, 0};
    if (live) {
        const double *cx = C.coef[0] + 8 * idx[0], *cy = C.coef[1] + 8 * idx[1], *cz = C.coef[2] + 8 * idx[2];
        Lx = D3{cx[0], 1.0, cx[1]}; Rx = D3{cx[2], cx[3], cx[4]};
        Ly = D3{cy[0], 1.0, cy[1]}; Ry = D3{cy[2], cy[3], cy[4]};
        Lz = D3{cz[0], 1.0, cz[1]}; Rz = D3{cz[2], cz[3], cz[4]};
    }
    if (live && lane < 27) {
        // window `lane`: direction d, cross offsets (s1, s2) along d1, d2
        WinList &R = wl[grp][lane];
        R.n = 0;
        int fb = 0;
        double minhb = 1.0;
        const int d = lane / 9, d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        const int s1 = (lane % 9) / 3 - 1, s2 = lane % 3 - 1;
        const D3 Ld = pick3(d, Lx, Ly, Lz), Rd = pick3(d, Rx, Ry, Rz);
        const double W = pick3(d1, Lx, Ly, Lz)[s1 + 1] * pick3(d2, Lx, Ly, Lz)[s2 + 1];
        int wc[3] = {0, 0, 0};
        wc[d1] = s1;
        wc[d2] = s2;
        bool sol[3];
        int nsol = 0;
        for (int p = -1; p <= 1; ++p) {
            int o[3] = {wc[0], wc[1], wc[2]};
            o[d] = p;
            size_t node = rownode + (ptrdiff_t)o[0] + (ptrdiff_t)o[1] * nx + (ptrdiff_t)o[2] * (ptrdiff_t)C.stride[2];
            sol[p + 1] = C.type[node] == 3;
            nsol += sol[p + 1];
        }
        if (nsol == 0) {
            for (int p = -1; p <= 1; ++p) {
                int o[3] = {wc[0], wc[1], wc[2]};
                o[d] = p;
                put(C, R, rownode, o, W * Rd[p + 1]);
            }
        } else if (nsol < 3) {      // a window inside the body is dropped
            int lo[2], hi[2], nr = 0;
            for (int p = -1; p <= 1;) {
                if (sol[p + 1]) { ++p; continue; }
                int a = p;
                while (p < 1 && !sol[p + 2]) ++p;
                lo[nr] = a;
                hi[nr] = p;
                ++nr;
                ++p;
            }
            const int pw = grp * 27 + lane;
            const PtBuf pb{pt_t[pw], pt_g[pw], pt_w[pw], pt_off[pw], pt_ibi[pw]};
            for (int q = 0; q < nr; ++q)
                run_operator(C, R, rownode, idx, d, wc, lo[q], hi[q], sol, nr, Ld, W, fb, minhb, bad, pb);
        }
        if (R.n > WIN_CAP) atomicOr(bad, 2);
        wfb[grp][lane] = fb;
        wminhb[grp][lane] = minhb;
    } else if (live && lane == 27) {
        // Q-bar: the row's L_x L_y L_z weights on f at every non-solid node of the 3x3x3 box
        double q = 0.0;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    size_t node = rownode + dx + (ptrdiff_t)dy * nx + (ptrdiff_t)dz * (ptrdiff_t)C.stride[2];
                    if (C.type[node] != 3) q += Lx[dx + 1] * Ly[dy + 1] * Lz[dz + 1] * C.f[node];
                }
        qbar[grp] = q;
        sw_krow(C, rownode, idx, k7 + 7 * (size_t)row);
    }
    __syncthreads();
    if (!live) return;
    // Sum the windows' lists in window order: lane l owns the slots l, l + 32, ... and adds
    // the entries for them in list order (the same order for every run) into its slots of
    // the row's LDS sums (a lane reads every entry's slot and only its own entries' values),
    // lane 0 the right-hand side, which starts from Q-bar.
    constexpr int SPL = (NSLOT + BR_LANES - 1) / BR_LANES;   // slots per lane
    double *sums = slot_sum[grp];
    uint32_t mused = 0u;
#pragma unroll
    for (int q = 0; q < SPL; ++q)
        if (lane + BR_LANES * q < NSLOT) sums[lane + BR_LANES * q] = 0.0;
    double rhs = qbar[grp];
    for (int w = 0; w < 27; ++w) {
        const WinList &R = wl[grp][w];
        const int n = min(R.n, WIN_CAP);
        for (int e = 0; e < n; ++e) {
            const int sl = R.slot[e];
            if (sl < 0) {
                if (lane == 0) rhs += R.v[e];
            } else if ((sl & (BR_LANES - 1)) == lane) {
                sums[sl] += R.v[e];
                mused |= 1u << (sl / BR_LANES);
            }
        }
    }
    double mine[SPL];
#pragma unroll
    for (int q = 0; q < SPL; ++q) mine[q] = lane + BR_LANES * q < NSLOT ? sums[lane + BR_LANES * q] : 0.0;
    // emit in slot order: slot sl = lane + 32 q; its output position is the number of used
    // slots before it (prefix over q, then over lanes)
    int cnt_total = 0, base_q = 0;
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
        const bool u = (mused >> q) & 1u;
        // used slots with the same q on lower lanes
        const uint64_t bal = __ballot(u);
        const uint64_t grpmask = (uint64_t)0xffffffffu << (BR_LANES * (threadIdx.x / BR_LANES % 2));
        const uint64_t mine_bits = bal & grpmask;
        const int before = __popcll(mine_bits & ((1ull << (threadIdx.x % 64)) - 1ull));
        const int here = __popcll(mine_bits);
        if (u) {
            const int sl = lane + BR_LANES * q;
            int o[3];
            if (sl < 27) {
                o[0] = sl % 3 - 1; o[1] = (sl / 3) % 3 - 1; o[2] = sl / 9 - 1;
            } else {
                int r2 = sl - 27;
                int t2 = r2 % 3 - 1; r2 /= 3;
                int t1 = r2 % 3 - 1; r2 /= 3;
                int m = r2 % 4 + 2; r2 /= 4;
                int pos = r2 % 2; int far = r2 / 2;
                o[far] = pos ? m : -m;
                o[(far + 1) % 3] = t1;
                o[(far + 2) % 3] = t2;
            }
            size_t node = rownode + (ptrdiff_t)o[0] + (ptrdiff_t)o[1] * nx + (ptrdiff_t)o[2] * (ptrdiff_t)C.stride[2];
            const int at = base_q + before;
            if (at < cap) {
                ell_col[(size_t)row * cap + at] = (int)node;
                ell_val[(size_t)row * cap + at] = mine[q];
            }
        }
        base_q += here;
        cnt_total = base_q;
    }
    if (lane == 13) bdiag[row] = mine[0];      // slot 13: the row's own node
    if (lane == 0) {
        int fb = 0;
        double minhb = 1.0;
        for (int w = 0; w < 27; ++w) {
            fb += wfb[grp][w];
            minhb = fmin(minhb, wminhb[grp][w]);
        }
        len[row] = min(cnt_total, cap);
        rhs_row[row] = rhs;
        minhb_row[row] = minhb;
        fb_row[row] = fb;
        if (cnt_total > cap) atomicOr(bad, 2);
    }
}

void launch_krows(hipStream_t s, int nx, int ny, int nz, const double *x, const double *y, const double *z,
                  const double *phi, const int8_t *type, int nirr, const int *nodes, double *k7)
{
    if (nirr == 0) return;
    Ctx C;
    C.n[0] = nx; C.n[1] = ny; C.n[2] = nz;
    C.stride[0] = 1; C.stride[1] = nx; C.stride[2] = (size_t)nx * ny;
    C.t[0] = x; C.t[1] = y; C.t[2] = z;
    for (int d = 0; d < 3; ++d) C.coef[d] = nullptr;
    C.phi = phi; C.g = phi; C.f = nullptr; C.type = type;   // g at an IBI is not used for K
    C.ibi_t = C.ibi_g = nullptr;
    C.irr_bits = nullptr;
    C.irr_wstart = nullptr;
    C.W = 0;
    k_krows<<<(unsigned)((8 * (size_t)nirr + 255) / 256), 256, 0, s>>>(C, nirr, nodes, k7);
}

void launch_gather3(hipStream_t s, int ncx, int ncy, int ncz, int nfx, int nfy, const int *ix, const int *iy,
                    const int *iz, const double *src, double *dst)
{
    k_gather3<<<dim3((unsigned)((ncx + 63) / 64), (unsigned)ncy, (unsigned)ncz), 64, 0, s>>>(ncx, ncy, ncz, nfx, nfy, ix,
                                                                                             iy, iz, src, dst);
}

void launch_build_rows(hipStream_t s, int nx, int ny, int nz, const double *x, const double *y, const double *z,
                       const double *coef, const double *phi, const double *g, const double *f, const int8_t *type,
                       int nirr, const int *nodes, const uint32_t *irr_bits, const int *irr_wstart, double *ibi_tab,
                       int cap, int *ell_col, double *ell_val, int *len, double *rhs_row, double *k7, double *bdiag,
                       double *minhb, int *fallback, int *bad)
{
    if (nirr == 0) return;
    Ctx C;
    C.n[0] = nx; C.n[1] = ny; C.n[2] = nz;
    C.stride[0] = 1; C.stride[1] = nx; C.stride[2] = (size_t)nx * ny;
    C.t[0] = x; C.t[1] = y; C.t[2] = z;
    int nmax = std::max(nx, std::max(ny, nz));
    for (int d = 0; d < 3; ++d) C.coef[d] = coef + (size_t)d * 8 * nmax;
    C.phi = phi; C.g = g; C.f = f; C.type = type;
    C.ibi_t = C.ibi_g = nullptr;
    C.irr_bits = irr_bits;
    C.irr_wstart = irr_wstart;
    C.W = (nx + 31) / 32;
    // every IBI next to an irregular node once, then the rows read them
    k_ibi_table<<<(unsigned)((6 * (size_t)nirr + 255) / 256), 256, 0, s>>>(C, nirr, nodes, ibi_tab,
                                                                          ibi_tab + 6 * (size_t)nirr);
    C.ibi_t = ibi_tab;
    C.ibi_g = ibi_tab + 6 * (size_t)nirr;
    k_build_rows<<<(nirr + BR_ROWS - 1) / BR_ROWS, BR_ROWS * BR_LANES, 0, s>>>(
        C, nirr, nodes, cap, ell_col, ell_val, len, rhs_row, k7, bdiag, minhb, fallback, bad);
}

// ELL scratch -> CSR: PACK_LANES consecutive lanes copy one row, so that each load and store
// of a wavefront covers contiguous entries of a few rows
constexpr int PACK_LANES = 16;
__global__ void __launch_bounds__(256) k_pack_rows(int nirr, int cap, const int *__restrict__ ell_col,
                                                   const double *__restrict__ ell_val, const int *__restrict__ len,
                                                   const int *__restrict__ ptr, int *__restrict__ col,
                                                   double *__restrict__ val64, float *__restrict__ val32)
{
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int row = t / PACK_LANES, l = t % PACK_LANES;
    if (row >= nirr) return;
    const int n = min(len[row], cap), o = ptr[row];
    const int *ec = ell_col + (size_t)row * cap;
    const double *ev = ell_val + (size_t)row * cap;
    for (int q = l; q < n; q += PACK_LANES) {
        col[o + q] = ec[q];
        const double v = ev[q];
        val64[o + q] = v;
        val32[o + q] = (float)v;
    }
}

void launch_pack_rows(hipStream_t s, int nirr, int cap, const int *ell_col, const double *ell_val, const int *len,
                      const int *ptr, int *col, double *val64, float *val32)
{
    if (nirr == 0) return;
    const size_t threads = (size_t)nirr * PACK_LANES;
    k_pack_rows<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(nirr, cap, ell_col, ell_val, len, ptr, col, val64,
                                                                  val32);
}

// ---------------------------------------------------------------------------------------
// right-hand side at regular rows: Q f (Eq. q) minus the known wall-node terms of Eq. A27
// ---------------------------------------------------------------------------------------
// Right-hand side of the regular rows: Q-bar f (the row's L_x L_y L_z weights on the 3 x 3 x 3
// box, Eq. q); k_rhs_walls then subtracts the terms of known wall neighbours (Eq. bc) at the
// rows next to a wall.  One wavefront covers 62
// consecutive nodes of an x-row (its two outer lanes only supply neighbours) in RHS_NK
// consecutive planes: each lane loads f at its own column in the three rows j - 1 .. j + 1 of
// the RHS_NK + 2 planes involved (all loads issued before any use), filters them along y once
// per plane and along z per output plane, and takes its x neighbours from the adjacent lanes.
// Blocks are numbered so that each XCD (blocks b = XCD mod NXCD) takes a contiguous range of
// z-chunks, whose halo planes its neighbours loaded into the same L2.
constexpr int RHS_SPAN = 62;
constexpr int RHS_NK = 8;
__global__ void __launch_bounds__(256) k_rhs_regular(int nx, int ny, int nz, const double *__restrict__ coef, int nmax,
                                                     const double *__restrict__ f, const double *__restrict__ g,
                                                     const int8_t *__restrict__ type, double *__restrict__ rhs,
                                                     int nbx, int nby, int total)
{
    const int per = (int)gridDim.x / NXCD;
    const int qb = ((int)blockIdx.x % NXCD) * per + (int)blockIdx.x / NXCD;
    if (qb >= total) return;
    const int bx = qb % nbx, by = (qb / nbx) % nby, bz = qb / (nbx * nby);
    const int lane = threadIdx.x;
    const int i = bx * RHS_SPAN + lane;                         // lanes 1..62 own nodes
    const int j = 1 + (int)(by * blockDim.y + threadIdx.y);
    const int k0 = 1 + bz * RHS_NK;
    if (j > ny - 2) return;                                     // whole wavefront
    const int nk = min(RHS_NK, nz - 1 - k0);                    // output planes k0 .. k0 + nk - 1
    const int ic = min(i, nx - 1);                              // lanes past the row read valid memory
    const size_t plane = (size_t)nx * ny;
    const size_t col = (size_t)ic + (size_t)nx * j;             // this lane's column, plane 0
    const double *cy = coef + 8 * (size_t)nmax + 8 * j;
    const double Ly[3] = {cy[0], 1.0, cy[1]};
    const double *cx = coef + 8 * ic;
    const double cx0 = cx[0], cx1 = cx[1];
    // f in rows j-1..j+1 of planes k0-1 .. k0+nk (clamped to the grid for a short last chunk)
    double fr3[RHS_NK + 2][3];
    int8_t te[RHS_NK];
#pragma unroll
    for (int p = 0; p < RHS_NK + 2; ++p) {
        const int kk = min(k0 - 1 + p, nz - 1);
#pragma unroll
        for (int q = 0; q < 3; ++q) fr3[p][q] = f[col + (ptrdiff_t)(q - 1) * nx + plane * kk];
    }
#pragma unroll
    for (int u = 0; u < RHS_NK; ++u) te[u] = type[col + plane * min(k0 + u, nz - 1)];
    // y-filtered f per plane: sum_q Ly[q] f(i, j+q-1, k)
    double fy[RHS_NK + 2];
#pragma unroll
    for (int p = 0; p < RHS_NK + 2; ++p) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc += Ly[q] * fr3[p][q];
        fy[p] = acc;
    }
    const bool own = lane >= 1 && lane <= RHS_SPAN && i <= nx - 2;
    const double Lx[3] = {cx0, 1.0, cx1};
#pragma unroll
    for (int u = 0; u < RHS_NK; ++u) {
        if (u >= nk) break;                                     // uniform over the wavefront
        const int k = k0 + u;
        const double *cz = coef + 16 * (size_t)nmax + 8 * k;
        const double Lz[3] = {cz[0], 1.0, cz[1]};
        double fyz = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) fyz += Lz[r] * fy[u + r];
        const double fl = __shfl_up(fyz, 1, 64), fr = __shfl_down(fyz, 1, 64);
        if (!own || te[u] != 1) continue;
        rhs[col + plane * k] = Lx[0] * fl + fyz + Lx[2] * fr;
    }
}

// The known (wall) neighbour terms of Eq. bc for the regular rows next to a wall, subtracted
// from the Q-bar f that k_rhs_regular stored, in the same order as a single pass would: a
// regular row has no solid neighbour, and the only other known nodes are the box walls, so a
// neighbour is known exactly when one of its indices is 0 or n - 1.  Face f = blockIdx.z
// (x-low, x-high, y-low, y-high, z-low, z-high) owns the interior nodes on it that no earlier
// face owns, so each such node is handled once.
__global__ void __launch_bounds__(256) k_rhs_walls(int nx, int ny, int nz, const double *__restrict__ coef, int nmax,
                                                   const double *__restrict__ g, const int8_t *__restrict__ type,
                                                   double *__restrict__ rhs)
{
    const int face = (int)blockIdx.z, u = (int)(blockIdx.x * blockDim.x + threadIdx.x), v = (int)blockIdx.y;
    int i, j, k;
    if (face < 2) {                     // i fixed; j = 1 + u, k = 1 + v
        i = face == 0 ? 1 : nx - 2; j = 1 + u; k = 1 + v;
        if (j > ny - 2 || k > nz - 2) return;
    } else if (face < 4) {              // j fixed; i = 2 + u, k = 1 + v
        j = face == 2 ? 1 : ny - 2; i = 2 + u; k = 1 + v;
        if (i > nx - 3 || k > nz - 2) return;
    } else {                            // k fixed; i = 2 + u, j = 2 + v
        k = face == 4 ? 1 : nz - 2; i = 2 + u; j = 2 + v;
        if (i > nx - 3 || j > ny - 3) return;
    }
    // a grid thinner than 3 interior points along an axis puts both faces on one plane
    if ((face == 1 && nx - 2 == 1) || (face == 3 && ny - 2 == 1) || (face == 5 && nz - 2 == 1)) return;
    const size_t plane = (size_t)nx * ny;
    const size_t e = (size_t)i + (size_t)nx * j + plane * k;
    if (type[e] != 1) return;
    const double *cx = coef + 8 * i, *cy = coef + 8 * (size_t)nmax + 8 * j, *cz = coef + 16 * (size_t)nmax + 8 * k;
    const double Lx[3] = {cx[0], 1.0, cx[1]}, Ly[3] = {cy[0], 1.0, cy[1]}, Lz[3] = {cz[0], 1.0, cz[1]};
    const double Rx[3] = {cx[2], cx[3], cx[4]}, Ry[3] = {cy[2], cy[3], cy[4]}, Rz[3] = {cz[2], cz[3], cz[4]};
    double acc = rhs[e];
    // every neighbour's g is loaded (no branch between the loads); a term that is not a
    // wall's subtracts 0 * g = 0 (g is finite), which leaves acc unchanged
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int ii = i + p - 1, jj = j + q - 1, kk = k + r - 1;
                const bool wall = ii == 0 || ii == nx - 1 || jj == 0 || jj == ny - 1 || kk == 0 || kk == nz - 1;
                const size_t nb = e + (p - 1) + (ptrdiff_t)(q - 1) * nx + (ptrdiff_t)(r - 1) * (ptrdiff_t)plane;
                const double a = Rx[p] * Ly[q] * Lz[r] + Lx[p] * Ry[q] * Lz[r] + Lx[p] * Ly[q] * Rz[r];
                acc -= (wall ? a : 0.0) * g[nb];
            }
    rhs[e] = acc;
}

void launch_rhs_regular(hipStream_t s, int nx, int ny, int nz, const double *coef, const double *f, const double *g,
                        const int8_t *type, double *rhs)
{
    if (nx < 3 || ny < 3 || nz < 3) return;
    int nmax = std::max(nx, std::max(ny, nz));
    const int nbx = (nx - 2 + RHS_SPAN - 1) / RHS_SPAN, nby = (ny - 2 + 3) / 4;
    const int nbz = (nz - 2 + RHS_NK - 1) / RHS_NK, total = nbx * nby * nbz;
    const int nb = (total + NXCD - 1) / NXCD * NXCD;
    k_rhs_regular<<<nb, dim3(64, 4), 0, s>>>(nx, ny, nz, coef, nmax, f, g, type, rhs, nbx, nby, total);
    const int fu = std::max(nx, ny), fv = std::max(ny, nz);
    k_rhs_walls<<<dim3((unsigned)((fu + 255) / 256), (unsigned)fv, 6), 256, 0, s>>>(nx, ny, nz, coef, nmax, g, type, rhs);
}

__global__ void k_scatter_rows(int nirr, const int *__restrict__ nodes, const double *__restrict__ rhs_row,
                               double *__restrict__ rhs)
{
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row < nirr) rhs[nodes[row]] = rhs_row[row];
}

void launch_scatter_rows(hipStream_t s, int nirr, const int *nodes, const double *rhs_row, double *rhs)
{
    if (nirr == 0) return;
    k_scatter_rows<<<(nirr + 255) / 256, 256, 0, s>>>(nirr, nodes, rhs_row, rhs);
}

__global__ void k_to_float(size_t n, const double *__restrict__ a, float *__restrict__ b)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        b[e] = (float)a[e];
}

void launch_to_float(hipStream_t s, size_t n, const double *a, float *b)
{
    if (n == 0) return;
    k_to_float<<<(unsigned)std::min<size_t>((n + 255) / 256, 65536), 256, 0, s>>>(n, a, b);
}

// min of a[] (starting from 1) and sum of fb[]: MINR_PARTS blocks write partials, then one
// block combines them (min and an integer sum do not depend on the order)
template <bool FINAL>
__global__ void __launch_bounds__(256) k_min_reduce(int n, const double *__restrict__ a, const long long *__restrict__ fb,
                                                    const int *__restrict__ fbi, double *out_min, long long *out_sum)
{
    __shared__ double smin[256];
    __shared__ long long ssum[256];
    double mn = 1.0;
    long long sm = 0;
    for (int q = (int)(blockIdx.x * blockDim.x + threadIdx.x); q < n; q += (int)(gridDim.x * blockDim.x)) {
        mn = fmin(mn, a[q]);
        sm += FINAL ? fb[q] : (long long)fbi[q];
    }
    smin[threadIdx.x] = mn;
    ssum[threadIdx.x] = sm;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
            ssum[threadIdx.x] += ssum[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_min[blockIdx.x] = smin[0];
        out_sum[blockIdx.x] = ssum[0];
    }
}

void launch_min_reduce(hipStream_t s, int n, const double *a, const int *fb, double *part, double *out_min,
                       long long *out_sum)
{
    double *pmin = part;
    long long *psum = (long long *)(part + MINR_PARTS);
    k_min_reduce<false><<<MINR_PARTS, 256, 0, s>>>(n, a, nullptr, fb, pmin, psum);
    k_min_reduce<true><<<1, 256, 0, s>>>(MINR_PARTS, pmin, psum, nullptr, out_min, out_sum);
}

// counts of the node types 0..3 (cnt[4], zeroed by the caller): 16 nodes per 16-byte load, a
// block sum per type and one atomic add per block and type
__global__ void __launch_bounds__(256) k_type_hist(size_t n, const int8_t *__restrict__ type, int *cnt)
{
    __shared__ int sh[4][4];
    int c[4] = {0, 0, 0, 0};
    const size_t n16 = n / 16;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n16; q += (size_t)gridDim.x * blockDim.x) {
        const int4 v = *reinterpret_cast<const int4 *>(type + 16 * q);
        const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int t = (w[u] >> (8 * b)) & 0xff;
                c[0] += t == 0; c[1] += t == 1; c[2] += t == 2; c[3] += t == 3;
            }
    }
    if (blockIdx.x == 0)
        for (size_t e = 16 * n16 + threadIdx.x; e < n; e += blockDim.x) {
            const int t = type[e];
            c[0] += t == 0; c[1] += t == 1; c[2] += t == 2; c[3] += t == 3;
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int v = c[t];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) sh[t][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int v = sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
        if (v) atomicAdd(cnt + threadIdx.x, v);
    }
}

void launch_type_hist(hipStream_t s, size_t n, const int8_t *type, int *cnt)
{
    const unsigned nb = (unsigned)std::min<size_t>((n / 16 + 255) / 256 + 1, 256);
    k_type_hist<<<nb, 256, 0, s>>>(n, type, cnt);
}

// ||b||^2 and ||D^-1 b||^2 over the unknowns (D = diag B): regular nodes take the diagonal
// from the 1D tables (sum of the three centre weights, as the apply kernels form it), the
// irregular rows their stored diagonal.  Per-block partials (2 per block) in a fixed order.
__global__ void __launch_bounds__(256) k_bnorms(int nx, int ny, int nz, const double *__restrict__ coef, int nmax,
                                                const int8_t *__restrict__ type, const double *__restrict__ b,
                                                int nirr, const int *__restrict__ nodes,
                                                const double *__restrict__ bdiag, double *__restrict__ partials)
{
    __shared__ double sh[2][4];
    double a0 = 0.0, a1 = 0.0;
    const double *cx = coef, *cy = coef + 8 * (size_t)nmax, *cz = coef + 16 * (size_t)nmax;
    for (int r = (int)blockIdx.x; r < ny * nz; r += (int)gridDim.x) {
        const int j = r % ny, k = r / ny;
        if (j < 1 || j > ny - 2 || k < 1 || k > nz - 2) continue;
        const size_t e0 = ((size_t)k * ny + j) * nx;
        const double dyz = cy[8 * j + 3], dz = cz[8 * k + 3];
        for (int i = 1 + (int)threadIdx.x; i <= nx - 2; i += (int)blockDim.x) {
            if (type[e0 + i] != 1) continue;
            const double v = b[e0 + i], rd = v / ((cx[8 * i + 3] + dyz) + dz);
            a0 += v * v;
            a1 += rd * rd;
        }
    }
    for (int q = (int)(blockIdx.x * blockDim.x + threadIdx.x); q < nirr; q += (int)(gridDim.x * blockDim.x)) {
        const double v = b[nodes[q]], rd = v / bdiag[q];
        a0 += v * v;
        a1 += rd * rd;
    }
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = a0;
        sh[1][threadIdx.x >> 6] = a1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
        partials[2 * blockIdx.x + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
    }
}

void launch_bnorms(hipStream_t s, int nx, int ny, int nz, const double *coef, const int8_t *type, const double *b,
                   int nirr, const int *nodes, const double *bdiag, double *partials, int nblocks)
{
    const int nmax = std::max(nx, std::max(ny, nz));
    k_bnorms<<<nblocks, 256, 0, s>>>(nx, ny, nz, coef, nmax, type, b, nirr, nodes, bdiag, partials);
}

}  // namespace cps
