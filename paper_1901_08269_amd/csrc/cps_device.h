// cps_device.h -- data layout and device helpers shared by the solver's HIP sources.
//
// Layout in HBM (node (i,j,k) at flat index i + nx*(j + ny*k), x fastest, walls included):
//   vectors        one full-grid array per Krylov vector, FP64 or FP32; wall and solid
//                  entries are kept at exactly 0 by every kernel (they are never written)
//   skip bits      one bit per node, 32 nodes per word along x, words (k*ny + j)*W + i/32;
//                  set for solid and irregular nodes: the tile kernels leave those rows to
//                  the irregular-row pass (irregular) or untouched (solid)
//   1D tables      per direction d and index n, 8 coefficients at coef[d][8n + q]:
//                  q = 0 a, 1 c, 2 ar, 3 br, 4 cr (compact scheme, Eq. app_xxx; b = 1),
//                  5 ka, 6 kb, 7 kc (second-order scheme of K, Eq. 2ndorder_coef)
//   irregular rows CSR over node indices (rows in increasing node order): the full row of
//                  B = A-bar + C (Eq. Bdec) at each irregular node, its 7-point K row and
//                  the diagonal entry of B
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace cps {

constexpr int TX = 64;        // tile width in x: one wavefront
constexpr int TY = 4;         // tile rows in y: one wavefront each
constexpr int NT = TX * TY;   // threads per block
constexpr int IRR_LANES = 16; // lanes per irregular row in the B pass
constexpr int NXCD = 8;       // MI355X: 8 XCDs, blocks dispatched round-robin over them
// rows per wavefront in the vectorised Chebyshev sweep: one row beats two (43.1 against
// 43.4 us per FP32 sweep at 256^3, with 1024 blocks instead of 512)
constexpr int RPW = 1;
// rows per wavefront of the sweeps that read two vectors (the first step of a smoothing pass,
// without an x_{k-1}, and the residual): they are bound by the latency of their plane steps,
// and two rows per wavefront put more bytes in flight per step
constexpr int RPW2 = 2;
// Vectors read by the vectorised sweeps carry this many zero elements past the last node:
// a lane always loads four consecutive elements, also where some lie past the row end.
constexpr size_t VEC_PAD = 8;

// A tiling of the interior into (tw x ty) columns that march over z-chunks of TZ planes.
struct Tiling {
    int tw;                    // tile width in x (nodes)
    int ty;                    // tile rows in y
    int tiles_x, tiles_y, zchunks, TZ;
    int ntiles;                // tiles_x * tiles_y * zchunks
    int nblk;                  // ntiles rounded up to a multiple of NXCD
};

struct Geom {
    int nx, ny, nz;
    int W;                     // skip-bit words per x-line
    Tiling ta;                 // 256 x 4 tiles, one row per wavefront: the B apply and the
                               // vector updates
    Tiling tr;                 // 256 x 4 tiles: one x-row segment of 256 nodes per wavefront,
                               // four nodes per lane (vectorised Chebyshev sweeps)
    Tiling tr2;                // 256 x (4 RPW2) tiles: RPW2 rows per wavefront (two-vector sweeps)
    Tiling tr2s;               // the same tiles in more z-chunks, for the FP32 two-vector sweeps
                               // (fewer registers: more of their wavefronts fit at once)
    int lg;                    // coarse multigrid levels whose rows are at most 128 nodes
                               // long: 2^lg lanes per row, 64 / 2^lg rows per wavefront
                               // (tr then has (4 * 2^lg) x (4 * 64 / 2^lg) tiles); 6 otherwise
    int nflat;                 // blocks of the flat (vectorised) pointwise kernels
};

template <typename T>
struct Coef {
    const T *c[3];
};

template <typename T>
struct Irr {
    int n;                     // irregular rows
    const int *node;           // node index of each row
    const int *ptr;            // CSR row pointer (n + 1)
    const int *col;            // node index of each entry (always an unknown)
    const T *val;              // B entries
    const T *k7;               // K row: diag, -x, +x, -y, +y, -z, +z
    const T *bdiag;            // diagonal entry of B
    const uint32_t *bits;      // irregular-node bits, laid out like the skip words
    const int *wstart;         // per bit word: rows of the nodes before the word's first node
};

// Row of irregular node (i, j, k) from its bit word: the rows are in node order, so the row
// is the word's start count plus the irregular nodes below i in that word.
template <typename T>
__device__ __forceinline__ int irr_row_of(const Irr<T> &ir, size_t word, int i)
{
    return ir.wstart[word] + __popc(ir.bits[word] & ((1u << (i & 31)) - 1u));
}

// Device-resident BiCGSTAB scalars (Alg. 1); all FP64 whatever the vector precision.
struct DevState {
    double rho;                // (r0, r_i)
    double alpha, omega, beta;
    double rn2s;               // recursive ||D^-1 r||^2 (D = diag B)
    double stop2;              // convergence threshold for rn2s
    double r0n2;               // ||r0||^2 (breakdown test)
    double res2, res2s;        // last true residual: ||r||^2 and ||D^-1 r||^2
    int done;                  // 0 running, 1 converged, 2 breakdown, 3 NaN
    int iters;                 // completed iterations
};

// the tiling of the two-vector sweeps in precision T
template <typename T>
__host__ __device__ __forceinline__ const Tiling &tr2_of(const Geom &g)
{
    return sizeof(T) == 4 ? g.tr2s : g.tr2;
}

__device__ __forceinline__ bool tile_of_block(const Tiling &t, int b, int &bx, int &by, int &bz)
{
    // Give each XCD a contiguous range of tiles so that the halos of neighbouring tiles
    // are served from the same L2.
    int per = t.nblk / NXCD;
    int q = (b % NXCD) * per + b / NXCD;
    if (q >= t.ntiles) return false;
    bx = q % t.tiles_x;
    q /= t.tiles_x;
    by = q % t.tiles_y;
    bz = q / t.tiles_y;
    return true;
}

__device__ __forceinline__ bool skip_bit(const uint32_t *skip, const Geom &g, int i, int j, int k)
{
    return (skip[((size_t)k * g.ny + j) * g.W + (i >> 5)] >> (i & 31)) & 1u;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block reduction of NV values over NT threads; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[NT / 64])
{
    int tid = threadIdx.x + threadIdx.y * blockDim.x;
    int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) sh[q][wv] = s;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += sh[q][w];
            v[q] = s;
        }
    }
}

// Writes this block's NV partial sums to partials[blockIdx.x * NV + q].  They are summed,
// in a fixed order, by a one-block finalize kernel launched next on the same stream: the
// kernel boundary makes every block's writes visible without device-scope fences.
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *partials)
{
    __shared__ double sh[NV][NT / 64];
    block_sum<NV>(v, sh);
    int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) partials[(size_t)blockIdx.x * NV + q] = v[q];
    }
}

// Fixed-order totals of the NV partial columns over nblocks blocks; valid in thread 0.
template <int NV>
__device__ __forceinline__ void total_partials(double (&tot)[NV], const double *partials, int nblocks)
{
    __shared__ double sh[NV][NT / 64];
    int tid = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int b = tid; b < nblocks; b += NT) s += partials[(size_t)b * NV + q];
        tot[q] = s;
    }
    block_sum<NV>(tot, sh);
}

}  // namespace cps
