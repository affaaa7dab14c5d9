// net.hip -- the learned warm start: a 4-level 3D convolutional encoder-decoder on the
// 4x-coarsened grid, trained on solutions that the solver itself produces.
//
// Network (channels c0..c3, 3 input channels f, phi, g; one output): per level two 3x3x3
// convolutions with bias and ReLU; 2x2x2 average pooling between encoder levels; nearest
// x2 upsampling and concatenation [upsampled, skip] on the way up; a 1x1x1 head.
// Parameters (FP32 master copy, flat): per 3x3x3 layer W[co][ci][kz][ky][kx] then b[co],
// in the order E0a E0b E1a E1b E2a E2b E3a E3b D2a D2b D1a D1b D0a D0b; then the head's
// c0 weights and its bias.
//
// Device layout: activations are BF16, voxel-major [b][z][y][x][C] with C a multiple of 16
// (the 3 input channels are zero-padded to 16).  3x3x3 weights are BF16 [co][tap][ci].
// Convolutions are implicit GEMMs on the matrix cores: v_mfma_f32_16x16x16bf16 with FP32
// accumulation; a wavefront computes 16 voxels x (16 NG) output channels.  The data
// gradient is the same kernel with tap-flipped, channel-transposed weights; the weight
// gradient is an MFMA GEMM over voxels with LDS-staged tiles and a fixed-order reduction
// over voxel chunks.  Gradients entering each 3x3x3 layer are rounded to BF16 (the MFMA
// operand type); everything else in the backward pass is FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "cps.h"
#include "cps_device.h"

namespace cpsnet {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

constexpr int NLAYER = 14;

__device__ __forceinline__ bf16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                 // round to nearest even
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x4 load4(const bf16 *p)
{
    return *reinterpret_cast<const bf16x4 *>(p);
}

// ---------------------------------------------------------------------------------------
// 3x3x3 convolution (zero padding): Y[v][co] = act(bias[co] + sum_{tap,ci} W[co][tap][ci] X[v+tap][ci])
// ---------------------------------------------------------------------------------------
template <int NG, bool RELU, bool BIAS, typename TO>
__global__ void __launch_bounds__(256) k_conv3(int n, int V, int Cin, int Cout, const bf16 *__restrict__ X,
                                               const bf16 *__restrict__ Wk, const float *__restrict__ bias,
                                               TO *__restrict__ Y)
{
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int v0 = wave * 16;
    if (v0 >= V) return;
    const int row = lane & 15, kq = lane >> 4;
    const int g0 = blockIdx.y * NG;
    const int n3 = n * n * n;
    const int v = v0 + row;
    const bool vin = v < V;
    int b = 0, z = 0, y = 0, x = 0;
    if (vin) {
        b = v / n3;
        int r = v - b * n3;
        z = r / (n * n);
        y = (r / n) % n;
        x = r % n;
    }
    f32x4 acc[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
    // The nine taps of one z-offset at a time: all their input and weight loads are issued
    // before the first of their MFMAs, so a wavefront waits for memory three times per
    // 16-channel slice instead of at every tap.  Sums run over (z-offset, channel slice, tap
    // in the plane): a fixed order.
    for (int tz = 0; tz < 3; ++tz) {
        const int zz = z + tz - 1;
        const bf16 *xp[9];
        bool ok[9];
#pragma unroll
        for (int t9 = 0; t9 < 9; ++t9) {
            const int yy = y + t9 / 3 - 1, xx = x + t9 % 3 - 1;
            ok[t9] = vin && zz >= 0 && yy >= 0 && xx >= 0 && zz < n && yy < n && xx < n;
            xp[t9] = X + (size_t)(b * n3 + (zz * n + yy) * n + xx) * Cin + 4 * kq;
        }
        for (int c0 = 0; c0 < Cin; c0 += 16) {
            bf16x4 a[9], w[9][NG];
#pragma unroll
            for (int t9 = 0; t9 < 9; ++t9) {
                a[t9] = ok[t9] ? load4(xp[t9] + c0) : bf16x4{0, 0, 0, 0};
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const int co = (g0 + g) * 16 + row;
                    w[t9][g] = load4(Wk + ((size_t)co * 27 + tz * 9 + t9) * Cin + c0 + 4 * kq);
                }
            }
#pragma unroll
            for (int t9 = 0; t9 < 9; ++t9)
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t9], w[t9][g], acc[g], 0, 0, 0);
        }
    }
    // D[voxel 4 kq + i][co = row]
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int co = (g0 + g) * 16 + row;
        const float bco = BIAS ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int vo = v0 + 4 * kq + i;
            if (vo >= V) continue;
            float val = acc[g][i] + bco;
            if (RELU) val = val > 0.f ? val : 0.f;
            if constexpr (sizeof(TO) == 2) Y[(size_t)vo * Cout + co] = f2bf(val);
            else Y[(size_t)vo * Cout + co] = val;
        }
    }
}

// ---------------------------------------------------------------------------------------
// weight gradient: P[chunk][co][tap][ci] = sum_{v in chunk} G[v][co] X[v+tap][ci]
// ---------------------------------------------------------------------------------------
// voxels per block: enough blocks to fill the GPU (about 2048 with the 27 taps), at most 4096
// voxels (fewer chunk partials to reduce), a multiple of WG_VS
inline int wgrad_chunk(int V)
{
    const int c = (int)std::min<long>(4096, std::max<long>(256, (long)V * 27 / 2048));
    return (c + 63) / 64 * 64;
}
constexpr int WG_VS = 64;        // voxels staged in LDS per barrier: four 16-voxel MFMA steps
constexpr int WG_MAXT = 7;       // 16x16 tiles per wave (Cout/16 * Cin/16 <= 28)

// A block stages WG_VS voxels of G and of the tap-shifted X at a time (8-byte loads).  With
// at least four 16x16 output tiles, wave w takes tiles w, w + 4, ... over all staged voxels;
// with fewer (the 16-channel layers, which run on the largest grids), wave w takes the w-th
// 16-voxel step of every tile and the four waves' sums are added in wave order at the end,
// so that no wave idles.
__global__ void __launch_bounds__(256) k_wgrad(int n, int V, int Cin, int Cout, int wchunk, const bf16 *__restrict__ G,
                                               const bf16 *__restrict__ X, float *__restrict__ P)
{
    __shared__ bf16 sG[WG_VS][64 + 4];
    __shared__ bf16 sX[WG_VS][112 + 4];
    __shared__ f32x4 red[3][3][64];
    const int tap = blockIdx.y, chunk = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n3 = n * n * n;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int tco = Cout / 16, tci = Cin / 16, ntiles = tco * tci;
    const bool split = ntiles < 4;
    f32x4 acc[WG_MAXT];
#pragma unroll
    for (int t = 0; t < WG_MAXT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int vbeg = chunk * wchunk, vend = min(vbeg + wchunk, V);
    const int g4 = Cout / 4, x4 = Cin / 4;
    const int m = lane & 15, kq = lane >> 4;
    for (int vs = vbeg; vs < vend; vs += WG_VS) {
        for (int q = tid; q < WG_VS * g4; q += 256) {
            const int r = q / g4, c = 4 * (q - r * g4), v = vs + r;
            const bf16x4 val = (v < vend) ? load4(G + (size_t)v * Cout + c) : bf16x4{0, 0, 0, 0};
            *reinterpret_cast<bf16x4 *>(&sG[r][c]) = val;
        }
        for (int q = tid; q < WG_VS * x4; q += 256) {
            const int r = q / x4, c = 4 * (q - r * x4), v = vs + r;
            bf16x4 val{0, 0, 0, 0};
            if (v < vend) {
                const int b = v / n3, rr = v - b * n3;
                const int z = rr / (n * n) + dz, y = (rr / n) % n + dy, x = rr % n + dx;
                if (z >= 0 && y >= 0 && x >= 0 && z < n && y < n && x < n)
                    val = load4(X + (size_t)(b * n3 + (z * n + y) * n + x) * Cin + c);
            }
            *reinterpret_cast<bf16x4 *>(&sX[r][c]) = val;
        }
        __syncthreads();
        for (int ks = 0; ks < WG_VS / 16; ++ks) {
            if (split && ks != wv) continue;
#pragma unroll
            for (int t = 0; t < WG_MAXT; ++t) {
                const int tile = split ? t : wv + 4 * t;
                if (tile >= ntiles) break;
                const int cog = tile / tci, cig = tile - cog * tci;
                bf16x4 a, bb;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    a[j] = (short)sG[16 * ks + 4 * kq + j][cog * 16 + m];    // A[co][v]
                    bb[j] = (short)sX[16 * ks + 4 * kq + j][cig * 16 + m];   // B[v][ci]
                }
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    if (split) {
        if (wv > 0)
            for (int t = 0; t < ntiles; ++t) red[wv - 1][t][lane] = acc[t];
        __syncthreads();
        if (wv > 0) return;
        for (int t = 0; t < ntiles; ++t)
            for (int w = 0; w < 3; ++w) acc[t] += red[w][t][lane];
    }
#pragma unroll
    for (int t = 0; t < WG_MAXT; ++t) {
        const int tile = split ? t : wv + 4 * t;
        if (tile >= ntiles) break;
        const int cog = tile / tci, cig = tile - cog * tci;
        for (int i = 0; i < 4; ++i) {
            const int co = cog * 16 + 4 * kq + i, ci = cig * 16 + m;   // D[co][ci]
            P[(((size_t)chunk * Cout + co) * 27 + tap) * Cin + ci] = acc[t][i];
        }
    }
}

// sum over chunks (fixed order) into the canonical gradient W[co][ci][tap] (ci < ci_real)
__global__ void k_wgrad_reduce(int nchunk, int Cin, int Cout, int ci_real, const float *__restrict__ P,
                               float *__restrict__ gW)
{
    // thread order (co, tap, ci): consecutive threads read consecutive partials of a chunk
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int total = Cout * ci_real * 27;
    if (q >= total) return;
    int ci = q % ci_real, tap = (q / ci_real) % 27, co = q / (27 * ci_real);
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += P[(((size_t)c * Cout + co) * 27 + tap) * Cin + ci];
    gW[((size_t)co * ci_real + ci) * 27 + tap] = s;
}

// db[c] = sum_v G[v][c] in two fixed-order passes.  Pass 1: COLSUM_BLOCKS blocks; thread t of
// a block takes channel t % C and every (256 / C)-th voxel of the block's stride (consecutive
// threads read consecutive elements), and the block sums its voxel lanes per channel in LDS
// in lane order.  Pass 2: one thread per channel adds the block partials in block order.
constexpr int COLSUM_BLOCKS = 512;
__global__ void __launch_bounds__(256) k_colsum_part(int V, int C, const bf16 *__restrict__ G, float *__restrict__ part)
{
    __shared__ float sh[256];
    const int lanes = 256 / C, t = (int)threadIdx.x;    // voxel lanes per block (C <= 256)
    const int c = t % C, vl = t / C;
    float s = 0.f;
    if (vl < lanes)
        for (size_t v = (size_t)blockIdx.x * lanes + vl; v < (size_t)V; v += (size_t)gridDim.x * lanes)
            s += bf2f(G[v * C + c]);
    sh[t] = s;
    __syncthreads();
    if (t < C) {
        float acc = 0.f;
        for (int l = 0; l < lanes; ++l) acc += sh[l * C + t];
        part[(size_t)blockIdx.x * C + t] = acc;
    }
}

// one block per channel: thread t adds partials t, t + 256, ...; then a tree in LDS
__global__ void __launch_bounds__(256) k_colsum_final(int nb, int C, const float *__restrict__ part,
                                                      float *__restrict__ out)
{
    __shared__ float sh[256];
    const int c = (int)blockIdx.x, t = (int)threadIdx.x;
    float acc = 0.f;
    for (int b = t; b < nb; b += 256) acc += part[(size_t)b * C + c];
    sh[t] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t == 0) out[c] = sh[0];
}

// ---------------------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------------------
// input [B][cin][n^3] (FP32, channels first) -> [V][16] BF16, channels >= cin zero
__global__ void k_pack_input(int V, int n3, int cin, const float *__restrict__ in, bf16 *__restrict__ out)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= V * 16) return;
    int v = q >> 4, c = q & 15;
    int b = v / n3, r = v - b * n3;
    out[q] = c < cin ? f2bf(in[((size_t)b * cin + c) * n3 + r]) : (bf16)0;
}

// 2x2x2 average pooling, [V][C] at n -> [V/8][C] at n/2
__global__ void k_pool(int B, int n, int C, const bf16 *__restrict__ in, bf16 *__restrict__ out)
{
    int m = n / 2;
    size_t total = (size_t)B * m * m * m * C;
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    int c = (int)(q % C);
    size_t v = q / C;
    int x = (int)(v % m), y = (int)((v / m) % m), z = (int)((v / ((size_t)m * m)) % m), b = (int)(v / ((size_t)m * m * m));
    float s = 0.f;
    for (int o = 0; o < 8; ++o) {
        int zz = 2 * z + (o >> 2), yy = 2 * y + ((o >> 1) & 1), xx = 2 * x + (o & 1);
        s += bf2f(in[((((size_t)b * n + zz) * n + yy) * n + xx) * C + c]);
    }
    out[q] = f2bf(s * 0.125f);
}

__global__ void k_pool_bwd(int B, int n, int C, const float *__restrict__ gout, float *__restrict__ gin)
{
    int m = n / 2;
    size_t total = (size_t)B * n * n * n * C;
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    int c = (int)(q % C);
    size_t v = q / C;
    int x = (int)(v % n), y = (int)((v / n) % n), z = (int)((v / ((size_t)n * n)) % n), b = (int)(v / ((size_t)n * n * n));
    gin[q] += gout[((((size_t)b * m + z / 2) * m + y / 2) * m + x / 2) * C + c] * 0.125f;
}

// [up(lo) (C0), skip (C1)] at n = 2m
__global__ void k_upcat(int B, int m, int C0, int C1, const bf16 *__restrict__ lo, const bf16 *__restrict__ skip,
                        bf16 *__restrict__ out)
{
    int n = 2 * m, C = C0 + C1;
    size_t total = (size_t)B * n * n * n * C;
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    int c = (int)(q % C);
    size_t v = q / C;
    if (c >= C0) {
        out[q] = skip[v * C1 + (c - C0)];
        return;
    }
    int x = (int)(v % n), y = (int)((v / n) % n), z = (int)((v / ((size_t)n * n)) % n), b = (int)(v / ((size_t)n * n * n));
    out[q] = lo[((((size_t)b * m + z / 2) * m + y / 2) * m + x / 2) * C0 + c];
}

// backward of k_upcat: glo[u][c] += sum of the 8 children; gskip[v][c] += g[v][C0 + c]
__global__ void k_upcat_bwd_lo(int B, int m, int C0, int C1, const float *__restrict__ g, float *__restrict__ glo)
{
    int n = 2 * m, C = C0 + C1;
    size_t total = (size_t)B * m * m * m * C0;
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    int c = (int)(q % C0);
    size_t u = q / C0;
    int x = (int)(u % m), y = (int)((u / m) % m), z = (int)((u / ((size_t)m * m)) % m), b = (int)(u / ((size_t)m * m * m));
    float s = 0.f;
    for (int o = 0; o < 8; ++o) {
        int zz = 2 * z + (o >> 2), yy = 2 * y + ((o >> 1) & 1), xx = 2 * x + (o & 1);
        s += g[((((size_t)b * n + zz) * n + yy) * n + xx) * C + c];
    }
    glo[q] += s;
}

__global__ void k_upcat_bwd_skip(size_t V, int C0, int C1, const float *__restrict__ g, float *__restrict__ gskip)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= V * C1) return;
    size_t v = q / C1;
    int c = (int)(q % C1);
    gskip[q] += g[v * (C0 + C1) + C0 + c];
}

__global__ void k_add(size_t n, const float *__restrict__ a, float *__restrict__ b)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) b[q] += a[q];
}

// gradient entering a 3x3x3 layer: ReLU mask of its output, rounded to BF16
__global__ void k_relu_bwd(size_t n, const float *__restrict__ g, const bf16 *__restrict__ act, bf16 *__restrict__ out)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = bf2f(act[q]) > 0.f ? f2bf(g[q]) : (bf16)0;
}

// head: p[v] = hb + sum_c hw[c] act[v][c]
__global__ void k_head(int V, int C, const bf16 *__restrict__ act, const float *__restrict__ hw, float *__restrict__ p)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    float s = hw[C];
    for (int c = 0; c < C; ++c) s += hw[c] * bf2f(act[(size_t)v * C + c]);
    p[v] = s;
}

// masked squared error: per-block partial sums of m (p - t)^2 and m
__global__ void k_loss_partial(int V, const float *__restrict__ p, const float *__restrict__ t,
                               const float *__restrict__ mask, double *__restrict__ part)
{
    __shared__ double s0[256], s1[256];
    double a = 0.0, w = 0.0;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < V; v += gridDim.x * 256) {
        double m = mask ? (double)mask[v] : 1.0;
        double d = (double)p[v] - (double)t[v];
        a += m * d * d;
        w += m;
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = w;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s0[threadIdx.x] += s0[threadIdx.x + o];
            s1[threadIdx.x] += s1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ void k_loss_final(int nb, const double *__restrict__ part, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, w = 0.0;
    for (int b = 0; b < nb; ++b) {
        a += part[2 * b];
        w += part[2 * b + 1];
    }
    out[0] = a / w;
    out[1] = w;
}

// head backward: dp = 2 m (p - t) / sum m; gact[v][c] = dp hw[c]; partials of dhw, dhb
constexpr int HEAD_BLOCKS = 512;    // blocks of the head's backward reduction
__global__ void k_head_bwd(int V, int C, const float *__restrict__ p, const float *__restrict__ t,
                           const float *__restrict__ mask, const double *__restrict__ lossw,
                           const bf16 *__restrict__ act, const float *__restrict__ hw, float *__restrict__ gact,
                           float *__restrict__ part /*[gridDim][C+1]*/)
{
    __shared__ float sh[256][17];
    const double inv = 1.0 / lossw[1];
    // C <= 16: the channel loops run over 16 with a guard, so that loc stays in registers
    float loc[17];
#pragma unroll
    for (int c = 0; c < 17; ++c) loc[c] = 0.f;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < V; v += gridDim.x * 256) {
        float m = mask ? mask[v] : 1.f;
        float dp = (float)(2.0 * m * ((double)p[v] - (double)t[v]) * inv);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            if (c >= C) break;
            float a = bf2f(act[(size_t)v * C + c]);
            gact[(size_t)v * C + c] = dp * hw[c];
            loc[c] += dp * a;
        }
        loc[16] += dp;
    }
#pragma unroll
    for (int c = 0; c < 16; ++c)
        if (c < C) sh[threadIdx.x][c] = loc[c];
    sh[threadIdx.x][C] = loc[16];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c <= C; ++c) sh[threadIdx.x][c] += sh[threadIdx.x + o][c];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c <= C; ++c) part[(size_t)blockIdx.x * (C + 1) + c] = sh[0][c];
}

// one block per output (C weights and the bias): partials t, t + 256, ... then a tree
__global__ void __launch_bounds__(256) k_head_bwd_final(int nb, int C, const float *__restrict__ part,
                                                        float *__restrict__ g)
{
    __shared__ float sh[256];
    const int c = (int)blockIdx.x, t = (int)threadIdx.x;
    float s = 0.f;
    for (int b = t; b < nb; b += 256) s += part[(size_t)b * (C + 1) + c];
    sh[t] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    if (t == 0) g[c] = sh[0];
}

// Adam on the FP32 master parameters (Kingma & Ba), step t >= 1
__global__ void k_adam(size_t n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2)
{
    size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    float gq = g[q];
    float a = b1 * m1[q] + (1.f - b1) * gq;
    float b = b2 * m2[q] + (1.f - b2) * gq * gq;
    m1[q] = a;
    m2[q] = b;
    w[q] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// pack canonical W[co][ci][tap] (FP32) into BF16 Wk[co][tap][cip] and flipped Wf[ci][tap'][co]
__global__ void k_pack_weights(int ci, int co, int cip, const float *__restrict__ W, bf16 *__restrict__ Wk,
                               bf16 *__restrict__ Wf)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= co * 27 * cip) return;
    int c = q % cip, tap = (q / cip) % 27, o = q / (27 * cip);
    float v = c < ci ? W[((size_t)o * ci + c) * 27 + tap] : 0.f;
    bf16 b = f2bf(v);
    Wk[q] = b;
    if (Wf && c < ci) Wf[((size_t)c * 27 + (26 - tap)) * co + o] = b;
}

// ---------------------------------------------------------------------------------------
// fine grid <-> coarse grid
// ---------------------------------------------------------------------------------------
// sums of g^2 and (f / 3 pi^2)^2 over all nodes (per-block partials; 1024 threads per
// block, 16-byte loads: a pass over two fine-grid FP64 arrays)
__global__ void __launch_bounds__(1024) k_scale_partial(size_t nn, const double *__restrict__ f,
                                                        const double *__restrict__ g, double *__restrict__ part)
{
    __shared__ double sh[1024];
    const double k = 1.0 / (3.0 * M_PI * M_PI);
    double s = 0.0;
    const size_t n2 = nn / 2;
    const double2 *f2 = reinterpret_cast<const double2 *>(f), *g2 = reinterpret_cast<const double2 *>(g);
    for (size_t e = (size_t)blockIdx.x * 1024 + threadIdx.x; e < n2; e += (size_t)gridDim.x * 1024) {
        const double2 a = g2[e], b = f2[e];
        const double b0 = b.x * k, b1 = b.y * k;
        s += (a.x * a.x + b0 * b0) + (a.y * a.y + b1 * b1);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (nn & 1)) {
        const double a = g[nn - 1], b = f[nn - 1] * k;
        s += a * a + b * b;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_scale_final(int nb, size_t nn, const double *__restrict__ part, double *__restrict__ sigma)
{
    if (threadIdx.x || blockIdx.x) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    double v = sqrt(s / (double)nn);
    sigma[0] = v > 0.0 ? v : 1.0;
}

// coarse cell (cx, cy, cz) <- means over fine interior nodes 1+4c .. 4+4c per direction:
// channel 0 f / (3 pi^2 sigma), 1 clamp(phi * nc / 8, -1, 1), 2 g / sigma; FP32 [1][3][nc^3]
__global__ void k_restrict(int nx, int ny, int nc, const double *__restrict__ f, const double *__restrict__ phi,
                           const double *__restrict__ g, const double *__restrict__ sigma, float *__restrict__ out)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int nc3 = nc * nc * nc;
    if (q >= nc3) return;
    int cx = q % nc, cy = (q / nc) % nc, cz = q / (nc * nc);
    double sf = 0.0, sp = 0.0, sg = 0.0;
    for (int dz = 0; dz < 4; ++dz)
        for (int dy = 0; dy < 4; ++dy)
            for (int dx = 0; dx < 4; ++dx) {
                size_t e = (size_t)(1 + 4 * cx + dx) + (size_t)nx * ((1 + 4 * cy + dy) + (size_t)ny * (1 + 4 * cz + dz));
                sf += f[e];
                sp += phi[e];
                sg += g[e];
            }
    const double inv = 1.0 / 64.0, s = sigma[0];
    out[q] = (float)(sf * inv / (3.0 * M_PI * M_PI * s));
    double ph = sp * inv * nc / 8.0;
    out[nc3 + q] = (float)(ph < -1.0 ? -1.0 : (ph > 1.0 ? 1.0 : ph));
    out[2 * nc3 + q] = (float)(sg * inv / s);
}

// target restriction: cell means over the same blocks of the solution's smooth extension
// (u at fluid nodes, g at nodes inside a body, phi <= 0), divided by sigma (FP32 [nc^3]).
// The solution itself is 0 inside the bodies; a cell mean that mixes those zeros with the
// fluid values interpolates badly next to the interface, where g continues u.
__global__ void k_restrict_u(int nx, int ny, int nc, const double *__restrict__ u, const double *__restrict__ phi,
                             const double *__restrict__ g, const double *__restrict__ sigma, float *__restrict__ out)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nc * nc * nc) return;
    int cx = q % nc, cy = (q / nc) % nc, cz = q / (nc * nc);
    double s = 0.0;
    for (int dz = 0; dz < 4; ++dz)
        for (int dy = 0; dy < 4; ++dy)
            for (int dx = 0; dx < 4; ++dx) {
                const size_t e =
                    (size_t)(1 + 4 * cx + dx) + (size_t)nx * ((1 + 4 * cy + dy) + (size_t)ny * (1 + 4 * cz + dz));
                s += phi[e] > 0.0 ? u[e] : g[e];
            }
    out[q] = (float)(s / 64.0 / sigma[0]);
}

// u0 at fine nodes: trilinear interpolation in index space of the coarse cell values
// (cell c centred at fine index 2.5 + 4c), constant beyond the outer cell centres
// one thread per node: x from the thread index, y and z from the grid (no index divisions)
__global__ void k_prolong(int nx, int ny, int nz, int nc, const float *__restrict__ p, const double *__restrict__ sigma,
                          double *__restrict__ u0)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x), j = (int)blockIdx.y, k = (int)blockIdx.z;
    if (i >= nx) return;
    const size_t e = (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k);
    int idx[3] = {i, j, k};
    int c0[3];
    float w[3];
    for (int d = 0; d < 3; ++d) {
        float s = ((float)idx[d] - 2.5f) * 0.25f;
        s = fminf(fmaxf(s, 0.f), (float)(nc - 1));
        int c = (int)floorf(s);
        if (c > nc - 2) c = nc - 2;
        if (c < 0) c = 0;
        c0[d] = c;
        w[d] = s - (float)c;
    }
    double acc = 0.0;
    for (int o = 0; o < 8; ++o) {
        int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        double ww = (ox ? w[0] : 1.f - w[0]) * (oy ? w[1] : 1.f - w[1]) * (oz ? w[2] : 1.f - w[2]);
        acc += ww * p[((c0[2] + oz) * nc + (c0[1] + oy)) * nc + (c0[0] + ox)];
    }
    u0[e] = acc * sigma[0];
}

}  // namespace cpsnet

// The sigma reduction of the restriction runs on SCALE_BLOCKS blocks whatever the grid size
// (grid-stride loop), so its scratch has a fixed size.
constexpr int SCALE_BLOCKS = 256;

// Scratch of cps_model_restrict_noalloc: [0, SCALE_BLOCKS) per-block partial sums of the
// sigma reduction, [SCALE_BLOCKS] sigma.  Every element is written before it is read in a
// call, so nothing needs clearing.  Each device holds one copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for that device.
static __device__ __align__(256) double scratch[SCALE_BLOCKS + 1];

// =========================================================================================
// model object and its C-ABI
// =========================================================================================
using namespace cpsnet;

// solver internals needed by the restriction (defined in solver.hip)
extern "C++" int cps_internal_fields(cps_solver *s, const double **phi, const double **g, const double **f, int *nx,
                                     int *ny, int *nz, void **stream);

struct LayerInfo {
    int ci, co, cip, lvl;
    long off;   // offset of W in the flat parameters (bias follows)
};

struct cps_model {
    cps_model_spec spec;
    hipStream_t stream = nullptr;
    LayerInfo L[NLAYER];
    long nparam = 0, head_off = 0;
    float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;   // flat FP32
    bf16 *Wk[NLAYER] = {}, *Wf[NLAYER] = {};
    bf16 *in[NLAYER] = {}, *out[NLAYER] = {};
    bool in_owned[NLAYER] = {};
    float *gout[NLAYER] = {};
    float *gtmp = nullptr;     // dgrad output (largest [V][ci])
    bf16 *gb = nullptr;        // BF16 masked gradient (largest [V][co])
    float *wpart = nullptr;    // weight-gradient chunk partials
    size_t wpart_n = 0;
    float *pred = nullptr, *tgt = nullptr, *msk = nullptr, *inp = nullptr;
    double *lpart = nullptr, *lossv = nullptr, *sig = nullptr;
    float *hpart = nullptr;
    float *cpart = nullptr;    // bias-gradient column-sum partials (COLSUM_BLOCKS x channels)
    int adam_t = 0;
    int device = 0;             // the device current at creation (its stream's device)
    std::vector<void *> allocs;
};

namespace {

struct NetFail {
    int code;
};

void nck(hipError_t e)
{
    if (e != hipSuccess) throw NetFail{CPS_EDEVICE};
}

inline unsigned nblk(size_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Device address of `scratch` on device `dev`, looked up once per device with that device
// current (the previous current device is restored).
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_dev[MAX_DEVICES] = {};

double *scratch_address(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) throw NetFail{CPS_EDEVICE};
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        int cur = 0;
        nck(hipGetDevice(&cur));
        if (cur != dev) nck(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) nck(hipSetDevice(cur));
        if (e != hipSuccess || !p) throw NetFail{CPS_EDEVICE};
        scratch_dev[dev] = static_cast<double *>(p);
    }
    return scratch_dev[dev];
}

// The network input of the solver's problem (and the target's cell means of u), with the
// sigma reduction's partial sums in part[SCALE_BLOCKS] and sigma in sig[0] (device).
// The network's inputs for the fields phi, g, f of an nx x ny x nz grid, queued on the
// model's stream; with `wait` the call returns once they are complete.
int restrict_fields(cps_model *m, int nx, int ny, int nz, const double *phi, const double *g, const double *f,
                    const double *u, float *inputs, float *target, double *sigma, double *part, double *sig, bool wait)
{
    const int nc = m->spec.nc;
    if (nx - 2 != 4 * nc || ny - 2 != 4 * nc || nz - 2 != 4 * nc || m->spec.in_ch != 3) return CPS_EINVAL;
    const size_t nn = (size_t)nx * ny * nz;
    k_scale_partial<<<SCALE_BLOCKS, 1024, 0, m->stream>>>(nn, f, g, part);
    k_scale_final<<<1, 64, 0, m->stream>>>(SCALE_BLOCKS, nn, part, sig);
    k_restrict<<<nblk((size_t)nc * nc * nc), 256, 0, m->stream>>>(nx, ny, nc, f, phi, g, sig, inputs);
    if (u && target)
        k_restrict_u<<<nblk((size_t)nc * nc * nc), 256, 0, m->stream>>>(nx, ny, nc, u, phi, g, sig, target);
    nck(hipGetLastError());
    if (sigma) nck(hipMemcpyAsync(sigma, sig, sizeof(double), hipMemcpyDeviceToHost, m->stream));
    if (wait) nck(hipStreamSynchronize(m->stream));
    return CPS_OK;
}

int restrict_into(cps_model *m, cps_solver *s, const double *u, float *inputs, float *target, double *sigma,
                  double *part, double *sig)
{
    const double *phi, *g, *f;
    int nx, ny, nz;
    void *sst;
    cps_internal_fields(s, &phi, &g, &f, &nx, &ny, &nz, &sst);
    return restrict_fields(m, nx, ny, nz, phi, g, f, u, inputs, target, sigma, part, sig, true);
}

template <typename T>
T *nalloc(cps_model *m, size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, (n ? n : 1) * sizeof(T)) != hipSuccess) throw NetFail{CPS_ENOMEM};
    m->allocs.push_back(p);
    nck(hipMemsetAsync(p, 0, (n ? n : 1) * sizeof(T), m->stream));
    return (T *)p;
}

void layer_table(const int ch[4], int cin, LayerInfo L[NLAYER])
{
    const int lv[NLAYER] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0};
    const int ci[NLAYER] = {cin, ch[0], ch[0], ch[1], ch[1], ch[2], ch[2], ch[3], ch[3] + ch[2], ch[2],
                            ch[2] + ch[1], ch[1], ch[1] + ch[0], ch[0]};
    const int co[NLAYER] = {ch[0], ch[0], ch[1], ch[1], ch[2], ch[2], ch[3], ch[3], ch[2], ch[2], ch[1], ch[1], ch[0], ch[0]};
    long off = 0;
    for (int q = 0; q < NLAYER; ++q) {
        L[q].ci = ci[q];
        L[q].co = co[q];
        L[q].cip = (ci[q] + 15) / 16 * 16;
        L[q].lvl = lv[q];
        L[q].off = off;
        off += (long)co[q] * ci[q] * 27 + co[q];
    }
}


int skip_of(int q) { return q == 8 ? 5 : (q == 10 ? 3 : 1); }

void launch_conv(cps_model *m, int n, int V, int Cin, int Cout, const bf16 *X, const bf16 *W, const float *bias, bool relu,
                 void *Y, bool fp32out)
{
    const int groups = Cout / 16;
    int NG = (groups % 4 == 0) ? 4 : (groups % 3 == 0) ? 3 : (groups % 2 == 0) ? 2 : 1;
    // A wavefront computes NG groups of 16 output channels from one load of its inputs.  On
    // the coarse levels (few voxels) that leaves most of the GPU idle, so there each
    // wavefront takes fewer groups and more blocks share the work (every output's sum runs
    // in the same order either way).
    const unsigned vblk = nblk((size_t)((V + 15) / 16) * 64);
    while (NG > 1 && (size_t)vblk * (groups / NG) < 1024) {
        int ng = NG - 1;
        while (groups % ng) --ng;
        NG = ng;
    }
    dim3 grid(vblk, groups / NG);
    hipStream_t s = m->stream;
#define CONV(NGv)                                                                                                    \
    if (NG == NGv) {                                                                                                 \
        if (fp32out)                                                                                                 \
            k_conv3<NGv, false, false, float><<<grid, 256, 0, s>>>(n, V, Cin, Cout, X, W, nullptr, (float *)Y);     \
        else if (relu)                                                                                               \
            k_conv3<NGv, true, true, bf16><<<grid, 256, 0, s>>>(n, V, Cin, Cout, X, W, bias, (bf16 *)Y);            \
        else                                                                                                         \
            k_conv3<NGv, false, true, bf16><<<grid, 256, 0, s>>>(n, V, Cin, Cout, X, W, bias, (bf16 *)Y);           \
    }
    CONV(1) CONV(2) CONV(3) CONV(4)
#undef CONV
}

void repack(cps_model *m)
{
    for (int q = 0; q < NLAYER; ++q) {
        const LayerInfo &l = m->L[q];
        k_pack_weights<<<nblk((size_t)l.co * 27 * l.cip), 256, 0, m->stream>>>(l.ci, l.co, l.cip, m->w + l.off, m->Wk[q],
                                                                               q > 0 ? m->Wf[q] : nullptr);
    }
}

void forward(cps_model *m, int B)
{
    const int nc = m->spec.nc;
    const int cin = m->spec.in_ch;
    int V0 = B * nc * nc * nc;
    k_pack_input<<<nblk((size_t)V0 * 16), 256, 0, m->stream>>>(V0, nc * nc * nc, cin, m->inp, m->in[0]);
    for (int q = 0; q < NLAYER; ++q) {
        const LayerInfo &l = m->L[q];
        const int n = nc >> l.lvl;
        const int V = B * n * n * n;
        if (q == 2 || q == 4 || q == 6) {
            k_pool<<<nblk((size_t)V * l.cip), 256, 0, m->stream>>>(B, 2 * n, l.cip, m->out[q - 1], m->in[q]);
        } else if (q == 8 || q == 10 || q == 12) {
            int sk = skip_of(q);
            k_upcat<<<nblk((size_t)V * l.cip), 256, 0, m->stream>>>(B, n / 2, m->L[q - 1].co, m->L[sk].co, m->out[q - 1],
                                                                    m->out[sk], m->in[q]);
        }
        launch_conv(m, n, V, l.cip, l.co, m->in[q], m->Wk[q], m->w + l.off + (long)l.co * l.ci * 27, true, m->out[q],
                    false);
    }
    k_head<<<nblk(V0), 256, 0, m->stream>>>(V0, m->L[NLAYER - 1].co, m->out[NLAYER - 1], m->w + m->head_off, m->pred);
}

void backward(cps_model *m, int B)
{
    const int nc = m->spec.nc;
    const int V0 = B * nc * nc * nc;
    const int C0 = m->L[NLAYER - 1].co;
    // loss
    const int nlb = 64;
    k_loss_partial<<<nlb, 256, 0, m->stream>>>(V0, m->pred, m->tgt, m->msk, m->lpart);
    k_loss_final<<<1, 64, 0, m->stream>>>(nlb, m->lpart, m->lossv);
    for (int q = 0; q < NLAYER; ++q) {
        const LayerInfo &l = m->L[q];
        const int n = nc >> l.lvl;
        nck(hipMemsetAsync(m->gout[q], 0, sizeof(float) * (size_t)B * n * n * n * l.co, m->stream));
    }
    const int nhb = HEAD_BLOCKS;
    k_head_bwd<<<nhb, 256, 0, m->stream>>>(V0, C0, m->pred, m->tgt, m->msk, m->lossv, m->out[NLAYER - 1],
                                           m->w + m->head_off, m->gout[NLAYER - 1], m->hpart);
    k_head_bwd_final<<<C0 + 1, 256, 0, m->stream>>>(nhb, C0, m->hpart, m->g + m->head_off);
    for (int q = NLAYER - 1; q >= 0; --q) {
        const LayerInfo &l = m->L[q];
        const int n = nc >> l.lvl;
        const int V = B * n * n * n;
        size_t nout = (size_t)V * l.co;
        k_relu_bwd<<<nblk(nout), 256, 0, m->stream>>>(nout, m->gout[q], m->out[q], m->gb);
        // weight and bias gradients
        const int wchunk = wgrad_chunk(V), nchunk = (V + wchunk - 1) / wchunk;
        k_wgrad<<<dim3(nchunk, 27), 256, 0, m->stream>>>(n, V, l.cip, l.co, wchunk, m->gb, m->in[q], m->wpart);
        k_wgrad_reduce<<<nblk((size_t)l.co * l.ci * 27), 256, 0, m->stream>>>(nchunk, l.cip, l.co, l.ci, m->wpart,
                                                                              m->g + l.off);
        k_colsum_part<<<COLSUM_BLOCKS, 256, 0, m->stream>>>(V, l.co, m->gb, m->cpart);
        k_colsum_final<<<l.co, 256, 0, m->stream>>>(COLSUM_BLOCKS, l.co, m->cpart,
                                                                 m->g + l.off + (long)l.co * l.ci * 27);
        if (q == 0) break;
        // data gradient into the producer of this layer's input
        launch_conv(m, n, V, l.co, l.cip, m->gb, m->Wf[q], nullptr, false, m->gtmp, true);
        if (q == 2 || q == 4 || q == 6) {
            size_t nin = (size_t)B * (2 * n) * (2 * n) * (2 * n) * l.cip;
            k_pool_bwd<<<nblk(nin), 256, 0, m->stream>>>(B, 2 * n, l.cip, m->gtmp, m->gout[q - 1]);
        } else if (q == 8 || q == 10 || q == 12) {
            int sk = skip_of(q);
            int C0u = m->L[q - 1].co, C1 = m->L[sk].co;
            size_t nlo = (size_t)B * (n / 2) * (n / 2) * (n / 2) * C0u;
            k_upcat_bwd_lo<<<nblk(nlo), 256, 0, m->stream>>>(B, n / 2, C0u, C1, m->gtmp, m->gout[q - 1]);
            k_upcat_bwd_skip<<<nblk((size_t)V * C1), 256, 0, m->stream>>>((size_t)V, C0u, C1, m->gtmp, m->gout[sk]);
        } else {
            k_add<<<nblk((size_t)V * l.ci), 256, 0, m->stream>>>((size_t)V * l.ci, m->gtmp, m->gout[q - 1]);
        }
    }
}

void free_model(cps_model *m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    for (void *p : m->allocs) (void)hipFree(p);
    delete m;
}

}  // namespace

extern "C" {

int64_t cps_model_param_count(const cps_model_spec *spec)
{
    if (!spec) return -1;
    LayerInfo L[NLAYER];
    layer_table(spec->channels, spec->in_ch, L);
    return L[NLAYER - 1].off + (long)L[NLAYER - 1].co * L[NLAYER - 1].ci * 27 + L[NLAYER - 1].co + spec->channels[0] + 1;
}

int cps_model_create(cps_model **out, const cps_model_spec *spec, void *stream)
{
    if (!out || !spec || spec->struct_size != (int32_t)sizeof(cps_model_spec)) return CPS_EINVAL;
    if (spec->nc < 8 || spec->nc % 8 || spec->batch < 1 || spec->in_ch < 1 || spec->in_ch > 16) return CPS_EINVAL;
    for (int q = 0; q < 4; ++q)
        if (spec->channels[q] < 16 || spec->channels[q] % 16 || spec->channels[q] > 64) return CPS_EINVAL;
    if (spec->channels[0] > 16) return CPS_EINVAL;   // the head reduction holds 16 channels
    *out = nullptr;
    cps_model *m = new (std::nothrow) cps_model();
    if (!m) return CPS_ENOMEM;
    m->spec = *spec;
    m->stream = (hipStream_t)stream;
    try {
        nck(hipGetDevice(&m->device));
        layer_table(spec->channels, spec->in_ch, m->L);
        m->head_off = m->L[NLAYER - 1].off + (long)m->L[NLAYER - 1].co * m->L[NLAYER - 1].ci * 27 + m->L[NLAYER - 1].co;
        m->nparam = m->head_off + spec->channels[0] + 1;
        m->w = nalloc<float>(m, m->nparam);
        m->g = nalloc<float>(m, m->nparam);
        m->m1 = nalloc<float>(m, m->nparam);
        m->m2 = nalloc<float>(m, m->nparam);
        const int B = spec->batch, nc = spec->nc;
        size_t maxci = 0, maxco = 0;
        for (int q = 0; q < NLAYER; ++q) {
            LayerInfo &l = m->L[q];
            const int n = nc >> l.lvl;
            const size_t V = (size_t)B * n * n * n;
            m->Wk[q] = nalloc<bf16>(m, (size_t)l.co * 27 * l.cip);
            if (q > 0) m->Wf[q] = nalloc<bf16>(m, (size_t)l.cip * 27 * l.co);
            m->out[q] = nalloc<bf16>(m, V * l.co);
            m->gout[q] = nalloc<float>(m, V * l.co);
            maxci = std::max(maxci, V * l.cip);
            maxco = std::max(maxco, V * l.co);
            // the chunk count for every batch size up to B (the chunk size depends on V)
            for (int bb = 1; bb <= B; ++bb) {
                const size_t Vb = (size_t)bb * n * n * n;
                const size_t wchunk = wgrad_chunk((int)Vb), nchunk = (Vb + wchunk - 1) / wchunk;
                m->wpart_n = std::max(m->wpart_n, nchunk * l.co * 27 * l.cip);
            }
        }
        for (int q = 0; q < NLAYER; ++q) {
            LayerInfo &l = m->L[q];
            const int n = nc >> l.lvl;
            const size_t V = (size_t)B * n * n * n;
            if (q == 0 || q == 2 || q == 4 || q == 6 || q == 8 || q == 10 || q == 12) {
                m->in[q] = nalloc<bf16>(m, V * l.cip);
                m->in_owned[q] = true;
            } else {
                m->in[q] = m->out[q - 1];
            }
        }
        m->gtmp = nalloc<float>(m, maxci);
        m->gb = nalloc<bf16>(m, maxco);
        m->wpart = nalloc<float>(m, m->wpart_n);
        const size_t V0 = (size_t)B * nc * nc * nc;
        m->pred = nalloc<float>(m, V0);
        m->tgt = nalloc<float>(m, V0);
        m->msk = nalloc<float>(m, V0);
        m->inp = nalloc<float>(m, V0 * spec->in_ch);
        m->lpart = nalloc<double>(m, 256);
        m->lossv = nalloc<double>(m, 2);
        m->sig = nalloc<double>(m, 1);
        m->hpart = nalloc<float>(m, HEAD_BLOCKS * 17);
        m->cpart = nalloc<float>(m, (size_t)COLSUM_BLOCKS * 64);   // channels are at most 64
        // He-normal initialisation from the spec's seed (host, deterministic)
        std::vector<float> h(m->nparam, 0.f);
        uint64_t st = spec->seed * 6364136223846793005ULL + 1442695040888963407ULL;
        auto unif = [&]() {
            st = st * 6364136223846793005ULL + 1442695040888963407ULL;
            return ((st >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        };
        for (int q = 0; q < NLAYER; ++q) {
            const LayerInfo &l = m->L[q];
            double sd = std::sqrt(2.0 / (27.0 * l.ci));
            for (long e = 0; e < (long)l.co * l.ci * 27; ++e)
                h[l.off + e] = (float)(sd * std::sqrt(-2.0 * std::log(unif())) * std::cos(2.0 * M_PI * unif()));
        }
        for (int c = 0; c < spec->channels[0]; ++c)
            h[m->head_off + c] = (float)(std::sqrt(1.0 / spec->channels[0]) * (2.0 * unif() - 1.0));
        nck(hipMemcpyAsync(m->w, h.data(), sizeof(float) * m->nparam, hipMemcpyHostToDevice, m->stream));
        repack(m);
        nck(hipStreamSynchronize(m->stream));
    } catch (NetFail &f) {
        free_model(m);
        return f.code;
    }
    *out = m;
    return CPS_OK;
}

int cps_model_set_params(cps_model *m, const float *params, int64_t n)
{
    if (!m || !params || n != m->nparam) return CPS_EINVAL;
    try {
        nck(hipMemcpyAsync(m->w, params, sizeof(float) * n, hipMemcpyHostToDevice, m->stream));
        nck(hipMemsetAsync(m->m1, 0, sizeof(float) * n, m->stream));
        nck(hipMemsetAsync(m->m2, 0, sizeof(float) * n, m->stream));
        m->adam_t = 0;
        repack(m);
        nck(hipStreamSynchronize(m->stream));
    } catch (NetFail &f) {
        return f.code;
    }
    return CPS_OK;
}

int cps_model_get_params(cps_model *m, float *params, float *grads, int64_t n)
{
    if (!m || n != m->nparam) return CPS_EINVAL;
    try {
        if (params) nck(hipMemcpyAsync(params, m->w, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream));
        if (grads) nck(hipMemcpyAsync(grads, m->g, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream));
        nck(hipStreamSynchronize(m->stream));
    } catch (NetFail &f) {
        return f.code;
    }
    return CPS_OK;
}

int cps_model_forward(cps_model *m, const float *inputs, int32_t batch, float *pred)
{
    if (!m || !inputs || !pred || batch < 1 || batch > m->spec.batch) return CPS_EINVAL;
    try {
        const size_t V0 = (size_t)batch * m->spec.nc * m->spec.nc * m->spec.nc;
        nck(hipMemcpyAsync(m->inp, inputs, sizeof(float) * V0 * m->spec.in_ch, hipMemcpyDeviceToDevice, m->stream));
        forward(m, batch);
        nck(hipMemcpyAsync(pred, m->pred, sizeof(float) * V0, hipMemcpyDeviceToDevice, m->stream));
        nck(hipStreamSynchronize(m->stream));
    } catch (NetFail &f) {
        return f.code;
    }
    return CPS_OK;
}

int cps_model_train_step(cps_model *m, const float *inputs, const float *target, const float *mask, int32_t batch,
                         float lr, int32_t update, double *loss_out)
{
    if (!m || !inputs || !target || batch < 1 || batch > m->spec.batch) return CPS_EINVAL;
    try {
        const size_t V0 = (size_t)batch * m->spec.nc * m->spec.nc * m->spec.nc;
        nck(hipMemcpyAsync(m->inp, inputs, sizeof(float) * V0 * m->spec.in_ch, hipMemcpyDeviceToDevice, m->stream));
        nck(hipMemcpyAsync(m->tgt, target, sizeof(float) * V0, hipMemcpyDeviceToDevice, m->stream));
        if (mask) nck(hipMemcpyAsync(m->msk, mask, sizeof(float) * V0, hipMemcpyDeviceToDevice, m->stream));
        forward(m, batch);
        float *keep = m->msk;
        if (!mask) m->msk = nullptr;
        backward(m, batch);
        m->msk = keep;
        if (update) {
            m->adam_t++;
            const float b1 = 0.9f, b2 = 0.999f;
            float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
            k_adam<<<nblk(m->nparam), 256, 0, m->stream>>>(m->nparam, m->w, m->g, m->m1, m->m2, lr, b1, b2, 1e-8f, c1, c2);
            repack(m);
        }
        double lv[2];
        nck(hipMemcpyAsync(lv, m->lossv, sizeof(double) * 2, hipMemcpyDeviceToHost, m->stream));
        nck(hipStreamSynchronize(m->stream));
        if (loss_out) *loss_out = lv[0];
    } catch (NetFail &f) {
        return f.code;
    }
    return CPS_OK;
}

int cps_model_restrict(cps_model *m, cps_solver *s, const double *u, float *inputs, float *target, double *sigma)
{
    if (!m || !s || !inputs) return CPS_EINVAL;
    try {
        return restrict_into(m, s, u, inputs, target, sigma, m->lpart, m->sig);
    } catch (NetFail &f_) {
        return f_.code;
    }
}

int cps_model_restrict_noalloc(cps_model *m, cps_solver *s, const double *u, float *inputs, float *target,
                               double *sigma)
{
    if (!m || !s || !inputs) return CPS_EINVAL;
    try {
        double *sp = scratch_address(m->device);
        return restrict_into(m, s, u, inputs, target, sigma, sp, sp + SCALE_BLOCKS);
    } catch (NetFail &f_) {
        return f_.code;
    }
}

int cps_model_predict(cps_model *m, cps_solver *s, double *u0)
{
    if (!m || !s || !u0) return CPS_EINVAL;
    const double *phi, *g, *f;
    int nx, ny, nz;
    void *sst;
    cps_internal_fields(s, &phi, &g, &f, &nx, &ny, &nz, &sst);
    const int nc = m->spec.nc;
    try {
        int rc = cps_model_restrict(m, s, nullptr, m->inp, nullptr, nullptr);
        if (rc) return rc;
        forward(m, 1);
        size_t nn = (size_t)nx * ny * nz;
        k_prolong<<<dim3(nblk((size_t)nx), (unsigned)ny, (unsigned)nz), 256, 0, m->stream>>>(nx, ny, nz, nc, m->pred,
                                                                                            m->sig, u0);
        nck(hipStreamSynchronize(m->stream));
    } catch (NetFail &f_) {
        return f_.code;
    }
    return CPS_OK;
}

int cps_model_predict_fields(cps_model *m, int32_t nx, int32_t ny, int32_t nz, const double *phi, const double *g,
                             const double *f, double *u0, void *stream)
{
    if (!m || !phi || !g || !f || !u0) return CPS_EINVAL;
    // the call's kernels go to `stream`; the model's own stream is restored on every return
    struct Restore {
        cps_model *m;
        hipStream_t st;
        ~Restore() { m->stream = st; }
    } restore{m, m->stream};
    if (stream) m->stream = (hipStream_t)stream;
    const int nc = m->spec.nc;
    try {
        int rc = restrict_fields(m, nx, ny, nz, phi, g, f, nullptr, m->inp, nullptr, nullptr, m->lpart, m->sig, false);
        if (rc) return rc;
        forward(m, 1);
        k_prolong<<<dim3(nblk((size_t)nx), (unsigned)ny, (unsigned)nz), 256, 0, m->stream>>>(nx, ny, nz, nc, m->pred,
                                                                                            m->sig, u0);
        nck(hipGetLastError());
    } catch (NetFail &f_) {
        return f_.code;
    }
    return CPS_OK;
}

namespace {

// File layout: 8-byte magic, the spec, nparam (long), then the FP32 weights; a checkpoint
// ("CPSNET02") adds the Adam step count (int64) and the two FP32 moment vectors.
int write_model(cps_model *m, const char *path, bool with_optimizer)
{
    if (!m || !path) return CPS_EINVAL;
    const size_t n = (size_t)m->nparam;
    std::vector<float> h(with_optimizer ? 3 * n : n);
    try {
        nck(hipMemcpyAsync(h.data(), m->w, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream));
        if (with_optimizer) {
            nck(hipMemcpyAsync(h.data() + n, m->m1, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream));
            nck(hipMemcpyAsync(h.data() + 2 * n, m->m2, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream));
        }
        nck(hipStreamSynchronize(m->stream));
    } catch (NetFail &f) {
        return f.code;
    }
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return CPS_EINVAL;
    const char *magic = with_optimizer ? "CPSNET02" : "CPSNET01";
    const int64_t t = m->adam_t;
    bool ok = std::fwrite(magic, 1, 8, fp) == 8 && std::fwrite(&m->spec, sizeof(m->spec), 1, fp) == 1 &&
              std::fwrite(&m->nparam, sizeof(m->nparam), 1, fp) == 1 &&
              (!with_optimizer || std::fwrite(&t, sizeof(t), 1, fp) == 1) &&
              std::fwrite(h.data(), sizeof(float), h.size(), fp) == h.size();
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? CPS_OK : CPS_EINVAL;
}

}  // namespace

int cps_model_save(cps_model *m, const char *path) { return write_model(m, path, false); }

int cps_model_save_checkpoint(cps_model *m, const char *path) { return write_model(m, path, true); }

int cps_model_load(cps_model *m, const char *path)
{
    if (!m || !path) return CPS_EINVAL;
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return CPS_EINVAL;
    char magic[8];
    cps_model_spec sp;
    long np = 0;
    int64_t t = 0;
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::fread(&sp, sizeof(sp), 1, fp) == 1 &&
              std::fread(&np, sizeof(np), 1, fp) == 1 && np == m->nparam;
    const bool ckpt = ok && std::memcmp(magic, "CPSNET02", 8) == 0;
    ok = ok && (ckpt || std::memcmp(magic, "CPSNET01", 8) == 0);
    if (ok && ckpt) ok = std::fread(&t, sizeof(t), 1, fp) == 1 && t >= 0 && t <= (int64_t)INT32_MAX;
    std::vector<float> h;
    if (ok) {
        h.resize(ckpt ? 3 * (size_t)np : (size_t)np);
        ok = std::fread(h.data(), sizeof(float), h.size(), fp) == h.size();
    }
    std::fclose(fp);
    if (!ok) return CPS_EINVAL;
    // the weights (and a fresh optimiser); a checkpoint then restores Adam's moments and step
    const int rc = cps_model_set_params(m, h.data(), np);
    if (rc != CPS_OK || !ckpt) return rc;
    try {
        nck(hipMemcpyAsync(m->m1, h.data() + np, sizeof(float) * np, hipMemcpyHostToDevice, m->stream));
        nck(hipMemcpyAsync(m->m2, h.data() + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice, m->stream));
        nck(hipStreamSynchronize(m->stream));
    } catch (NetFail &f) {
        return f.code;
    }
    m->adam_t = (int)t;
    return CPS_OK;
}

void cps_model_destroy(cps_model *m) { free_model(m); }

}  // extern "C"
