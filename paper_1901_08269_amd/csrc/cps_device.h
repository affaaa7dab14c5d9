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

namespace cps {

constexpr int TX = 64;        // tile width in x: one wavefront
constexpr int TY = 4;         // tile rows in y: one wavefront each
constexpr int NT = TX * TY;   // threads per block
constexpr int IRR_LANES = 16; // lanes per irregular row in the B pass
constexpr int NXCD = 8;       // MI355X: 8 XCDs, blocks dispatched round-robin over them

struct Geom {
    int nx, ny, nz;
    int W;                     // skip-bit words per x-line
    int tiles_x, tiles_y, zchunks, TZ;
    int ntiles;                // tiles_x * tiles_y * zchunks
    int nblk_tiles;            // ntiles rounded up to a multiple of NXCD
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
};

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

__device__ __forceinline__ bool tile_of_block(const Geom &g, int b, int &bx, int &by, int &bz)
{
    // Give each XCD a contiguous range of tiles so that the halos of neighbouring tiles
    // are served from the same L2.
    int per = g.nblk_tiles / NXCD;
    int t = (b % NXCD) * per + b / NXCD;
    if (t >= g.ntiles) return false;
    bx = t % g.tiles_x;
    t /= g.tiles_x;
    by = t % g.tiles_y;
    bz = t / g.tiles_y;
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

// Writes this block's partial sums; returns true in every thread of the block that
// finishes last.  That block then reads all partials (fixed order) and resets the ticket.
template <int NV>
__device__ __forceinline__ bool publish_partials(double (&v)[NV], double *partials, unsigned *ticket, int nblocks)
{
    __shared__ double sh[NV > 0 ? NV : 1][NT / 64];
    __shared__ bool last;
    block_sum<NV>(v, sh);
    int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) partials[(size_t)blockIdx.x * NV + q] = v[q];
        __threadfence();
        unsigned t = atomicAdd(ticket, 1u);
        last = (t == (unsigned)nblocks - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// In the last block: totals of the NV partial columns in fixed order; valid in thread 0.
template <int NV>
__device__ __forceinline__ void total_partials(double (&tot)[NV], const double *partials, unsigned *ticket, int nblocks)
{
    __shared__ double sh[NV > 0 ? NV : 1][NT / 64];
    int tid = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int b = tid; b < nblocks; b += NT) s += partials[(size_t)b * NV + q];
        tot[q] = s;
    }
    block_sum<NV>(tot, sh);
    if (tid == 0) *ticket = 0u;
}

}  // namespace cps
