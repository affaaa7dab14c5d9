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
__global__ void k_coef(int n, const double *__restrict__ t, double *__restrict__ coef)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double *o = coef + 8 * (size_t)i;
    for (int q = 0; q < 8; ++q) o[q] = 0.0;
    if (i == 0 || i == n - 1) {
        // wall indices: never used by a row; nonzero diagonals keep flat pointwise
        // kernels finite on the (zero) wall entries
        o[3] = -1.0;
        o[6] = -1.0;
        return;
    }
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

void launch_coef(hipStream_t s, int n, const double *t, double *coef)
{
    k_coef<<<(n + 255) / 256, 256, 0, s>>>(n, t, coef);
}

// ---------------------------------------------------------------------------------------
// classification
// ---------------------------------------------------------------------------------------
// one thread per node: x from the thread index, y and z from the grid (no 64-bit divisions)
__global__ void __launch_bounds__(256) k_classify(int nx, int ny, int nz, const double *__restrict__ phi,
                                                  const double *__restrict__ g, const double *__restrict__ f,
                                                  int8_t *__restrict__ type, int *flags)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int j = (int)(blockIdx.y * blockDim.y + threadIdx.y);
    const int k = (int)blockIdx.z;
    if (i >= nx || j >= ny) return;
    const size_t e = (size_t)i + (size_t)nx * j + (size_t)nx * ny * k;
    const double p = phi[e];
    if (!isfinite(p) || !isfinite(g[e]) || !isfinite(f[e])) atomicOr(flags, 1);
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
                     int8_t *type, int *flags)
{
    dim3 blk(64, 4), grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4), (unsigned)nz);
    k_classify<<<grid, blk, 0, s>>>(nx, ny, nz, phi, g, f, type, flags);
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
constexpr int CMP_THREADS = 256, CMP_PER_THREAD = 16, CMP_CHUNK = CMP_THREADS * CMP_PER_THREAD;

int compact_blocks(size_t n) { return (int)((n + CMP_CHUNK - 1) / CMP_CHUNK); }

__global__ void k_count(size_t n, const int8_t *__restrict__ type, int8_t want, int *blockcnt)
{
    __shared__ int sh[CMP_THREADS];
    size_t base = (size_t)blockIdx.x * CMP_CHUNK + (size_t)threadIdx.x * CMP_PER_THREAD;
    int c = 0;
    for (int q = 0; q < CMP_PER_THREAD; ++q)
        if (base + q < n && type[base + q] == want) ++c;
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
    int c = 0;
    for (int q = 0; q < CMP_PER_THREAD; ++q)
        if (base + q < n && type[base + q] == want) ++c;
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
    for (int q = 0; q < CMP_PER_THREAD; ++q)
        if (base + q < n && type[base + q] == want) list[pos++] = (int)(base + q);
}

// exclusive scan of n ints by one block; out[n] = total
__global__ void k_scan(const int *__restrict__ in, int *__restrict__ out, int n)
{
    __shared__ int sh[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        int idx = base + threadIdx.x;
        int v = idx < n ? in[idx] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int a = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (idx < n) out[idx] = carry + sh[threadIdx.x] - v;
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

// One-sided weights on NP points (coordinates pt) that reproduce sum over the run of
// Ld[p] u''(x_p) for every polynomial of degree < NP: the moment conditions in coordinates
// scaled by the reference point tref and the largest offset href.
template <int NP>
__device__ __forceinline__ bool onesided_weights(const double *pt, const double *tr, int plo, int phi_, const double Ld[3],
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
constexpr int PT_CAP = 8;
struct PtBuf {
    double *t, *g, *w;
    signed char *off;
    bool *ibi;
};

// one fluid run [plo, phi_] (positions -1..1 along d of the window centred at `wc` = row
// offset) of a window meeting the body
__device__ __forceinline__ void run_operator(const Ctx &C, WinList &R, size_t rownode, const int rowidx[3], int d, const int wc[3],
                             int plo, int phi_, const bool sol[3], int nruns, const double Ld[3], double W, int &fb,
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
        P.t[np] = t;
        P.off[np] = (signed char)off;
        P.ibi[np] = ibi;
        P.g[np] = gv;
        ++np;
    };
    bool shortened = false;
    double gv, fr;
    if (sl && sr) {
        double tl = ibi_on_segment(C, d, line0, cidx + plo, cidx + plo - 1, &gv, &fr);
        minhb = fmin(minhb, fr);
        push(tl, 0, true, gv);
        for (int p = plo; p <= phi_; ++p) push(C.t[d][cidx + p], p, false, 0.0);
        double th = ibi_on_segment(C, d, line0, cidx + phi_, cidx + phi_ + 1, &gv, &fr);
        minhb = fmin(minhb, fr);
        push(th, 0, true, gv);
        shortened = true;
    } else {
        const int want = (nruns == 2) ? 5 : 6;
        for (int p = plo; p <= phi_; ++p) push(C.t[d][cidx + p], p, false, 0.0);
        int near = sr ? phi_ : plo;                 // run node next to the interface
        int step = sr ? -1 : 1;                     // march away from the interface
        double tb = ibi_on_segment(C, d, line0, cidx + near, cidx + near - step, &gv, &fr);
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
                double te = ibi_on_segment(C, d, line0, cidx + pos, gi, &gv, &fr);
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
        if (C.type[nm] == 3) hb = C.t[d][idx[d]] - ibi_on_segment(C, d, line0, idx[d], idx[d] - 1, &gv, &fr);
        if (C.type[npl] == 3) hf = ibi_on_segment(C, d, line0, idx[d], idx[d] + 1, &gv, &fr) - C.t[d][idx[d]];
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
    __shared__ double pt_t[BR_ROWS * BR_LANES][PT_CAP], pt_g[BR_ROWS * BR_LANES][PT_CAP],
        pt_w[BR_ROWS * BR_LANES][PT_CAP];
    __shared__ signed char pt_off[BR_ROWS * BR_LANES][PT_CAP];
    __shared__ bool pt_ibi[BR_ROWS * BR_LANES][PT_CAP];
    __shared__ double qbar[BR_ROWS];
    __shared__ int wfb[BR_ROWS][27];
    __shared__ double wminhb[BR_ROWS][27];
    const int grp = threadIdx.x / BR_LANES, lane = threadIdx.x % BR_LANES;
    const int row = blockIdx.x * BR_ROWS + grp;
    const bool live = row < nirr;
    const size_t rownode = live ? (size_t)nodes[row] : 0;
    const int nx = C.n[0], ny = C.n[1];
    const int idx[3] = {(int)(rownode % nx), (int)((rownode / nx) % ny), (int)(rownode / ((size_t)nx * ny))};
    double L[3][3], Rr[3][3];
    if (live) {
        for (int d = 0; d < 3; ++d) {
            const double *c = C.coef[d] + 8 * idx[d];
            L[d][0] = c[0]; L[d][1] = 1.0; L[d][2] = c[1];
            Rr[d][0] = c[2]; Rr[d][1] = c[3]; Rr[d][2] = c[4];
        }
    }
    if (live && lane < 27) {
        // window `lane`: direction d, cross offsets (s1, s2) along d1, d2
        WinList &R = wl[grp][lane];
        R.n = 0;
        int fb = 0;
        double minhb = 1.0;
        const int d = lane / 9, d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        const int s1 = (lane % 9) / 3 - 1, s2 = lane % 3 - 1;
        const double W = L[d1][s1 + 1] * L[d2][s2 + 1];
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
                put(C, R, rownode, o, W * Rr[d][p + 1]);
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
            const PtBuf pb{pt_t[threadIdx.x], pt_g[threadIdx.x], pt_w[threadIdx.x], pt_off[threadIdx.x],
                           pt_ibi[threadIdx.x]};
            for (int q = 0; q < nr; ++q)
                run_operator(C, R, rownode, idx, d, wc, lo[q], hi[q], sol, nr, L[d], W, fb, minhb, bad, pb);
        }
        if (R.n > WIN_CAP) atomicOr(bad, 2);
        wfb[grp][lane] = fb;
        wminhb[grp][lane] = minhb;
    } else if (live && lane == 27) {
        // Q-bar: the row's L_x L_y L_z weights on f at every non-solid node of the 3x3x3 box
        double q = 0.0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    size_t node = rownode + dx + (ptrdiff_t)dy * nx + (ptrdiff_t)dz * (ptrdiff_t)C.stride[2];
                    if (C.type[node] != 3) q += L[0][dx + 1] * L[1][dy + 1] * L[2][dz + 1] * C.f[node];
                }
        qbar[grp] = q;
        sw_krow(C, rownode, idx, k7 + 7 * (size_t)row);
    }
    __syncthreads();
    if (!live) return;
    // Sum the windows' lists in window order: lane l owns the slots l, l + 32, ... and adds
    // the entries for them in list order (the same order for every run), lane 0 the
    // right-hand side, which starts from Q-bar.
    constexpr int SPL = (NSLOT + BR_LANES - 1) / BR_LANES;   // slots per lane
    double mine[SPL];
    uint32_t mused = 0u;
    for (int q = 0; q < SPL; ++q) mine[q] = 0.0;
    double rhs = qbar[grp];
    for (int w = 0; w < 27; ++w) {
        const WinList &R = wl[grp][w];
        const int n = min(R.n, WIN_CAP);
        for (int e = 0; e < n; ++e) {
            const int sl = R.slot[e];
            if (sl < 0) {
                if (lane == 0) rhs += R.v[e];
            } else if (sl % BR_LANES == lane) {
                mine[sl / BR_LANES] += R.v[e];
                mused |= 1u << (sl / BR_LANES);
            }
        }
    }
    // emit in slot order: slot sl = lane + 32 q; its output position is the number of used
    // slots before it (prefix over q, then over lanes)
    int cnt_total = 0, base_q = 0;
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
                       int nirr, const int *nodes, int cap, int *ell_col, double *ell_val, int *len, double *rhs_row,
                       double *k7, double *bdiag, double *minhb, int *fallback, int *bad)
{
    if (nirr == 0) return;
    Ctx C;
    C.n[0] = nx; C.n[1] = ny; C.n[2] = nz;
    C.stride[0] = 1; C.stride[1] = nx; C.stride[2] = (size_t)nx * ny;
    C.t[0] = x; C.t[1] = y; C.t[2] = z;
    int nmax = std::max(nx, std::max(ny, nz));
    for (int d = 0; d < 3; ++d) C.coef[d] = coef + (size_t)d * 8 * nmax;
    C.phi = phi; C.g = g; C.f = f; C.type = type;
    k_build_rows<<<(nirr + BR_ROWS - 1) / BR_ROWS, BR_ROWS * BR_LANES, 0, s>>>(
        C, nirr, nodes, cap, ell_col, ell_val, len, rhs_row, k7, bdiag, minhb, fallback, bad);
}

__global__ void k_pack_rows(int nirr, int cap, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                            const int *__restrict__ len, const int *__restrict__ ptr, int *__restrict__ col,
                            double *__restrict__ val64, float *__restrict__ val32)
{
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nirr) return;
    int n = min(len[row], cap), o = ptr[row];
    for (int q = 0; q < n; ++q) {
        col[o + q] = ell_col[(size_t)row * cap + q];
        double v = ell_val[(size_t)row * cap + q];
        val64[o + q] = v;
        val32[o + q] = (float)v;
    }
}

void launch_pack_rows(hipStream_t s, int nirr, int cap, const int *ell_col, const double *ell_val, const int *len,
                      const int *ptr, int *col, double *val64, float *val32)
{
    if (nirr == 0) return;
    k_pack_rows<<<(nirr + 255) / 256, 256, 0, s>>>(nirr, cap, ell_col, ell_val, len, ptr, col, val64, val32);
}

// ---------------------------------------------------------------------------------------
// right-hand side at regular rows: Q f (Eq. q) minus the known wall-node terms of Eq. A27
// ---------------------------------------------------------------------------------------
// Right-hand side of the regular rows: Q-bar f (the row's L_x L_y L_z weights on the 3 x 3 x 3
// box, Eq. q) minus the terms of known wall neighbours (Eq. bc).  One wavefront covers 62
// consecutive nodes of an x-row (its two outer lanes only supply neighbours): each lane
// loads f at its own node in the nine rows of the box and takes its x neighbours from the
// adjacent lanes, so f is read 9 instead of 27 times per node.
constexpr int RHS_SPAN = 62;
__global__ void __launch_bounds__(256) k_rhs_regular(int nx, int ny, int nz, const double *__restrict__ coef, int nmax,
                                                     const double *__restrict__ f, const double *__restrict__ g,
                                                     const int8_t *__restrict__ type, double *__restrict__ rhs)
{
    const int lane = threadIdx.x;
    const int i = (int)blockIdx.x * RHS_SPAN + lane;            // lanes 1..62 own nodes
    const int j = 1 + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    const int k = 1 + (int)blockIdx.z;
    if (j > ny - 2) return;                                     // whole wavefront
    const int ic = min(i, nx - 1);                              // lanes past the row read valid memory
    const size_t plane = (size_t)nx * ny;
    const size_t e = (size_t)ic + (size_t)nx * j + plane * k;
    const double *cy = coef + 8 * (size_t)nmax + 8 * j, *cz = coef + 16 * (size_t)nmax + 8 * k;
    const double Ly[3] = {cy[0], 1.0, cy[1]}, Lz[3] = {cz[0], 1.0, cz[1]};
    // y and z filtered f at this lane's column: sum_{q,r} Ly[q] Lz[r] f(i, j+q-1, k+r-1)
    double fyz = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc += Ly[q] * f[e + (ptrdiff_t)(q - 1) * nx + (ptrdiff_t)(r - 1) * (ptrdiff_t)plane];
        fyz += Lz[r] * acc;
    }
    const double fl = __shfl_up(fyz, 1, 64), fr = __shfl_down(fyz, 1, 64);
    const bool own = lane >= 1 && lane <= RHS_SPAN && i <= nx - 2;
    if (!own || type[e] != 1) return;
    const double *cx = coef + 8 * i;
    const double Lx[3] = {cx[0], 1.0, cx[1]};
    double acc = Lx[0] * fl + fyz + Lx[2] * fr;
    // known (wall) neighbours move to the right-hand side; only rows next to a wall have them
    // (a regular row has no solid neighbour)
    if (i == 1 || j == 1 || k == 1 || i == nx - 2 || j == ny - 2 || k == nz - 2) {
        const double Rx[3] = {cx[2], cx[3], cx[4]}, Ry[3] = {cy[2], cy[3], cy[4]}, Rz[3] = {cz[2], cz[3], cz[4]};
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q)
                for (int p = 0; p < 3; ++p) {
                    const size_t nb = e + (p - 1) + (ptrdiff_t)(q - 1) * nx + (ptrdiff_t)(r - 1) * (ptrdiff_t)plane;
                    if (type[nb] == 0) {
                        const double a = Rx[p] * Ly[q] * Lz[r] + Lx[p] * Ry[q] * Lz[r] + Lx[p] * Ly[q] * Rz[r];
                        acc -= a * g[nb];
                    }
                }
    }
    rhs[e] = acc;
}

void launch_rhs_regular(hipStream_t s, int nx, int ny, int nz, const double *coef, const double *f, const double *g,
                        const int8_t *type, double *rhs)
{
    if (nx < 3 || ny < 3 || nz < 3) return;
    int nmax = std::max(nx, std::max(ny, nz));
    dim3 blk(64, 4), grid((unsigned)((nx - 2 + RHS_SPAN - 1) / RHS_SPAN), (unsigned)((ny - 2 + 3) / 4), (unsigned)(nz - 2));
    k_rhs_regular<<<grid, blk, 0, s>>>(nx, ny, nz, coef, nmax, f, g, type, rhs);
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

// min of a[] and sum of fb[] by one block
__global__ void k_min_reduce(int n, const double *__restrict__ a, const int *__restrict__ fb, double *out_min,
                             long long *out_sum)
{
    __shared__ double smin[256];
    __shared__ long long ssum[256];
    double mn = 1.0;
    long long sm = 0;
    for (int q = threadIdx.x; q < n; q += 256) {
        mn = fmin(mn, a[q]);
        sm += fb[q];
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
        *out_min = smin[0];
        *out_sum = ssum[0];
    }
}

void launch_min_reduce(hipStream_t s, int n, const double *a, const int *fb, double *out_min, long long *out_sum)
{
    k_min_reduce<<<1, 256, 0, s>>>(n, a, fb, out_min, out_sum);
}

}  // namespace cps
