// multigrid.hip -- grid transfers of the multigrid preconditioner for K.
//
// The paper preconditions BiCGSTAB with the second-order operator K (Sec. 3.3) applied
// approximately by an inner solver, and allows other inner solvers than its own.  The
// multigrid inner solver is one V-cycle on a hierarchy of grids: a coarser grid keeps, along
// every axis, the even-indexed points and the last one, and carries its own K built from the
// level set at its nodes.  Prolongation P is the tensor product of 1D linear interpolation
// in the physical coordinate; restriction is P^T with every coarse row divided by its sum.
// Both act on unknown nodes only: every other node holds 0 on every level; the coarse
// correction is added at the regular unknown nodes (not at the irregular ones).
//
// 1D tables per axis (built on the host from the coordinates):
//   prolongation  for each fine index i, whose left coarse index is a = min(i / 2, nc - 2):
//                 the weight w[i] of coarse node a + 1 (fine value = (1 - w) e[a] +
//                 w e[a + 1]); the weights carry 4 zeros of padding
//   restriction   for each interior coarse index I (fine point 2I): the weights rw[3I + q]
//                 of fine points 2I - 1 + q, q = 0 .. 2, already divided by the row sum
#include <hip/hip_runtime.h>

#include "cps_kernels.h"

namespace cps {

namespace {

__device__ __forceinline__ bool unknown(int8_t t) { return t == 1 || t == 2; }

template <typename T>
struct MgVec4;
template <>
struct MgVec4<float> {
    typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct MgVec4<double> {
    typedef double type __attribute__((ext_vector_type(4), aligned(8)));
};

// Coarse rho(I, J, K) = sum over the 3 x 3 x 3 fine nodes (2I - 1 .. 2I + 1, ...) of
// rwx rwy rwz r at the unknown coarse nodes, 0 at the other interior nodes (the walls of rc
// are never written and stay 0).  Block 64 x 4: lane l takes the interior coarse nodes
// I0 = 1 + 128 blockIdx.x + 2 l and I0 + 1 of row J = 1 + 4 blockIdx.y + wavefront, plane
// K = 1 + blockIdx.z; it reads fine nodes 2 I0 - 1 .. 2 I0 + 2 of each of the nine fine
// rows as a 4-vector, and node 2 I0 + 3 from the next lane.  Every load is issued whatever
// the node types.
// With a first step F (F.x1 non-null) it also writes the coarse level's first Chebyshev
// step from zero, x1 = c2 rho / diag K, at its unknown nodes.
template <typename T>
__global__ void __launch_bounds__(256) k_mg_restrict(int ncx, int ncy, int nfx, int nfy, MgAxis<T> ax, MgAxis<T> ay,
                                                     MgAxis<T> az, const T *__restrict__ r, T *__restrict__ rc,
                                                     MgFirst<T> F)
{
    using V = typename MgVec4<T>::type;
    const int I0 = 1 + (int)(blockIdx.x * 128 + 2 * threadIdx.x), J = 1 + (int)(blockIdx.y * 4 + threadIdx.y);
    const int K = 1 + (int)blockIdx.z;
    if (I0 > ncx - 2 || J > ncy - 2) return;
    const bool two = I0 + 1 <= ncx - 2;
    const int I1 = two ? I0 + 1 : I0;
    T w0[3], w1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w0[a] = ax.rw[3 * I0 + a];
        w1[a] = ax.rw[3 * I1 + a];
    }
    const size_t ec = (size_t)I0 + (size_t)ncx * (J + (size_t)ncy * K);
    const T dg0 = F.diag[ec], dg1 = two ? F.diag[ec + 1] : T(0);
    const bool unk0 = dg0 != T(0), unk1 = dg1 != T(0);
    const size_t fplane = (size_t)nfx * nfy;
    const int f0 = 2 * I0 - 1;                      // first fine node of the lane
    const int f4 = min(f0 + 4, nfx - 1);            // fifth node (I0 + 1's last), in the row
    // the fifth node is the next lane's first one, taken by a shuffle unless that lane has no
    // coarse node (then the lane loads it)
    const bool self4 = threadIdx.x == 63 || I0 + 2 > ncx - 2;
    T acc0 = T(0), acc1 = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T wz = az.rw[3 * K + c];
        const size_t kz = (size_t)(2 * K - 1 + c) * fplane;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T wyz = wz * ay.rw[3 * J + b];
            const T *row = r + kz + (size_t)(2 * J - 1 + b) * nfx;
            const V v = *reinterpret_cast<const V *>(row + f0);
            T v4 = __shfl_down(v.x, 1, 64);
            if (self4) v4 = row[f4];
            acc0 += wyz * (w0[0] * v.x + w0[1] * v.y + w0[2] * v.z);
            acc1 += wyz * (w1[0] * v.z + w1[1] * v.w + w1[2] * v4);
        }
    }
    rc[ec] = unk0 ? acc0 : T(0);
    if (two) rc[ec + 1] = unk1 ? acc1 : T(0);
    if (F.x1) {
        if (unk0) F.x1[ec] = F.c2 * acc0 / dg0;
        if (unk1) F.x1[ec + 1] = F.c2 * acc1 / dg1;
    }
}

// A wave-uniform value moved to a scalar register.
__device__ __forceinline__ float wave_uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// rho - K x at a regular node from its seven x values (centre c, then the -x, +x, -y, +y,
// -z, +z neighbours) and the 1D tables of its three indices (Eq. 2ndorder_coef).
template <typename T>
__device__ __forceinline__ T mg_reg_resid(T rh, T c, T w, T e, T s, T n, T m, T u, T kax, T kbx, T kcx, T kay,
                                          T kby, T kcy, T za, T zb, T zc)
{
    const T kd = kbx + kby + zb;
    return rh - (kd * c + kax * w + kcx * e + kay * s + kcy * n + za * m + zc * u);
}

// Residual and restriction in one pass on the problem's grid: rc = R (rho - K x) at the
// unknown coarse nodes, 0 at the other interior ones (the sums of k_mg_restrict, in its
// order), with no fine residual stored.  A wavefront owns coarse row J of a 128-node coarse
// segment bs and the coarse planes K0 .. K1 - 1 of a chunk.  Lane l takes coarse nodes
// I0 = 1 + 128 bs + 2 l and I0 + 1, whose fine points are f0 = 2 I0 - 1 .. f0 + 4: it forms
// the residual at f0 .. f0 + 3 (the four-node layout of the vectorised sweeps) and takes
// the one at f0 + 4 from the next lane; the last lane forms its own fifth node when its
// segment owns I0 + 1 and f0 + 4 is interior.  The wavefront marches over the fine planes
// 2 K0 - 1 .. 2 K1 - 1: at each it forms the residual of fine rows 2J - 1 .. 2J + 1 from x
// on rows 2J - 2 .. 2J + 2 (the planes below and above carried in registers), combines it
// in x and y, and adds it to the coarse planes that the fine plane belongs to; coarse plane
// K is complete, and stored, after fine plane 2K + 1.  Fine rows 2J - 1 and 2J + 1 are formed
// by both wavefronts that need them, the first fine plane of a chunk by both chunks.
// Irregular and solid fine nodes (skip bits) take their residual from ri, which holds it
// at the irregular nodes (the irregular rows of the residual kernel, run before) and 0 at
// the solid ones; walls give 0.  With a first step F (F.x1 non-null) the coarse level's first Chebyshev
// step from zero is written too, as k_mg_restrict does.
// Loads through a buffer resource based at a wave-uniform address (one plane of an
// array): the 32-bit byte offset of each lane goes in a vector register and the base in
// scalar registers, so an address costs no 64-bit vector arithmetic (this kernel issues
// about twenty loads per plane step, and its throughput is bound by instruction issue).
typedef uint32_t MgU4 __attribute__((ext_vector_type(4)));
struct MgF4 {
    float v[4];
};
struct MgD2 {
    double v[2];
};
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base)
{
    // raw buffer (stride 0), range 4 GiB from the base, 32-bit data format (CDNA)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, 0x00020000);
}
template <typename T>
__device__ __forceinline__ typename MgVec4<T>::type bload4(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ MgVec4<float>::type bload4<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const MgF4 f = __builtin_bit_cast(MgF4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    return MgVec4<float>::type{f.v[0], f.v[1], f.v[2], f.v[3]};
}
template <>
__device__ __forceinline__ MgVec4<double>::type bload4<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const MgD2 a = __builtin_bit_cast(MgD2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    const MgD2 b = __builtin_bit_cast(MgD2, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0));
    return MgVec4<double>::type{a.v[0], a.v[1], b.v[0], b.v[1]};
}
template <typename T>
__device__ __forceinline__ T bload1(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bload1<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double bload1<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ uint32_t bload_u32(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

template <typename T, bool FIFTH, int CR>
__global__ void __launch_bounds__(256) k_mg_resid_restrict(Geom g, Tiling tl, Coef<T> cf,
                                                           const uint32_t *__restrict__ skip,
                                                           const T *__restrict__ x, const T *__restrict__ rho,
                                                           const T *__restrict__ ri, int ncx, int ncy, int ncz,
                                                           MgAxis<T> ax, MgAxis<T> ay, MgAxis<T> az,
                                                           T *__restrict__ rc, MgFirst<T> F, const DevState *st)
{
    constexpr int NR = 2 * CR + 1;                            // fine residual rows of a wavefront
    using V = typename MgVec4<T>::type;
    if (st && st->done) return;
    int bs, by, bz;
    if (!tile_of_block(tl, (int)blockIdx.x, bs, by, bz)) return;
    const int J0 = 1 + (by * 4 + (int)threadIdx.y) * CR;     // the wavefront's first coarse row
    if (J0 > ncy - 2) return;                                  // whole wavefront
    const int lane = (int)threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t plane = (size_t)nx * ny, wplane = (size_t)ny * g.W;
    const int I0 = 1 + 128 * bs + 2 * lane;
    const bool own0 = I0 <= ncx - 2, own1 = I0 + 1 <= ncx - 2;
    const int f0 = 2 * I0 - 1;
    const int nv = min(4, nx - 1 - f0);                       // interior fine nodes of the lane
    // the lane's loads start at node ic: f0, or the wall node for lanes past the row end.
    // Values past the lane's valid nodes are never used: their residuals are zeroed, and
    // the +x neighbour of the last interior node is the wall node (0 in every vector).
    const int ic = min(f0, nx - 1);
    const bool need5 = FIFTH && lane == 63 && own1 && f0 + 4 <= nx - 2;
    const bool needl = lane == 0 && bs > 0;                   // node f0 - 1 is interior
    // the skip bits that matter: the lane's interior nodes, and the fifth node where formed
    const uint32_t smask = ((1u << max(nv, 0)) - 1u) | (need5 ? 0x10u : 0u);
    T w0[3], w1[3];
    {
        const int a0 = own0 ? I0 : 1, a1 = own1 ? I0 + 1 : a0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            w0[a] = ax.rw[3 * a0 + a];
            w1[a] = ax.rw[3 * a1 + a];
        }
    }
    T kax[5], kbx[5], kcx[5];
#pragma unroll
    for (int u = 0; u < 5; ++u) {
        const bool ok = u < 4 ? u < nv : need5;
        const T *cx = cf.c[0] + 8 * (ok ? f0 + u : 1);
        kax[u] = cx[5];
        kbx[u] = cx[6];
        kcx[u] = cx[7];
    }
    // in-plane byte offsets of node ic on x rows 2 J0 - 2 .. 2 J0 + 2 CR (clamped to the wall
    // row, where x is 0); the residual rows 2 J0 - 1 .. 2 J0 + 2 CR - 1 are x rows 1 .. NR,
    // those past the last interior row zeroed; ow: byte offsets of their skip words
    uint32_t ox[NR + 2], ow[NR];
#pragma unroll
    for (int c = 0; c < NR + 2; ++c) ox[c] = (uint32_t)((ic + nx * min(2 * J0 - 2 + c, ny - 1)) * sizeof(T));
    bool rok[NR];
    T kay[NR], kby[NR], kcy[NR];
#pragma unroll
    for (int b = 0; b < NR; ++b) {
        const int j = 2 * J0 - 1 + b;
        rok[b] = j <= ny - 2;
        const int jc = min(j, ny - 1);
        ow[b] = (uint32_t)((jc * g.W + (ic >> 5)) * sizeof(uint32_t));
        kay[b] = wave_uniform(cf.c[1][8 * jc + 5]);
        kby[b] = wave_uniform(cf.c[1][8 * jc + 6]);
        kcy[b] = wave_uniform(cf.c[1][8 * jc + 7]);
    }
    // the coarse rows J0 .. J0 + CR - 1 (those past the last interior one are not stored)
    // and their y weights on fine rows 2J - 1 .. 2J + 1
    bool jok[CR];
    T wy[CR][3];
#pragma unroll
    for (int c = 0; c < CR; ++c) {
        jok[c] = J0 + c <= ncy - 2;
#pragma unroll
        for (int q = 0; q < 3; ++q) wy[c][q] = jok[c] ? wave_uniform(ay.rw[3 * (J0 + c) + q]) : T(0);
    }

    const int K0 = 1 + bz * tl.TZ, K1 = min(K0 + tl.TZ, ncz - 1);
    const int p0 = 2 * K0 - 1, p1 = 2 * K1 - 1;
    // x of the residual rows at the plane below (m) and at the current one (c); the fifth
    // node's in m5, c5
    V xm[NR], xc[NR];
    T m5[NR], c5[NR];
    {
        const __amdgpu_buffer_rsrc_t xb = plane_rsrc(x + (size_t)(p0 - 1) * plane), x0 = plane_rsrc(x + (size_t)p0 * plane);
#pragma unroll
        for (int b = 0; b < NR; ++b) {
            xm[b] = bload4<T>(xb, ox[b + 1]);
            xc[b] = bload4<T>(x0, ox[b + 1]);
            m5[b] = need5 ? bload1<T>(xb, ox[b + 1] + 4 * sizeof(T)) : T(0);
            c5[b] = need5 ? bload1<T>(x0, ox[b + 1] + 4 * sizeof(T)) : T(0);
        }
    }
    // the coarse plane being summed: the diagonals of its nodes (0 where not an unknown),
    // loaded when the plane opens and used when it is stored two fine planes later
    T acc0[CR], acc1[CR], dg0[CR], dg1[CR];
#pragma unroll
    for (int c = 0; c < CR; ++c) acc0[c] = acc1[c] = dg0[c] = dg1[c] = T(0);
    auto coarse_at = [&](int c, int K) -> size_t {
        return (size_t)(own0 ? I0 : 1) + (size_t)ncx * (min(J0 + c, ncy - 2) + (size_t)ncy * K);
    };
    auto open = [&](int K) {
#pragma unroll
        for (int c = 0; c < CR; ++c) {
            acc0[c] = T(0);
            acc1[c] = T(0);
            const size_t ec = coarse_at(c, K);
            dg0[c] = (own0 && jok[c]) ? F.diag[ec] : T(0);
            dg1[c] = (own1 && jok[c]) ? F.diag[ec + 1] : T(0);
        }
    };
    auto emit = [&](int K) {
#pragma unroll
        for (int c = 0; c < CR; ++c) {
            if (!jok[c]) continue;
            const size_t ec = coarse_at(c, K);
            if (own0) rc[ec] = dg0[c] != T(0) ? acc0[c] : T(0);
            if (own1) rc[ec + 1] = dg1[c] != T(0) ? acc1[c] : T(0);
            if (F.x1) {
                if (dg0[c] != T(0)) F.x1[ec] = F.c2 * acc0[c] / dg0[c];
                if (dg1[c] != T(0)) F.x1[ec + 1] = F.c2 * acc1[c] / dg1[c];
            }
        }
    };
    // coarse plane K += its z weight q times the fine plane's rows, restricted in y
    auto add_plane = [&](int K, int q, const T *xr0, const T *xr1) {
        const T wz = wave_uniform(az.rw[3 * K + q]);
#pragma unroll
        for (int c = 0; c < CR; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T wyz = wz * wy[c][b];
                acc0[c] += wyz * xr0[2 * c + b];
                acc1[c] += wyz * xr1[2 * c + b];
            }
    };
    // skip bits of nodes ic .. ic + 4 on the residual rows of plane q (words read in pairs;
    // the array carries two words of padding), loaded one plane ahead
    auto skip_bits = [&](int q, int b) -> uint32_t {
        const __amdgpu_buffer_rsrc_t sq = plane_rsrc(skip + (size_t)q * wplane);
        const uint64_t pair = (uint64_t)bload_u32(sq, ow[b]) | ((uint64_t)bload_u32(sq, ow[b] + 4) << 32);
        return (uint32_t)(pair >> (ic & 31)) & smask;
    };
    uint32_t skn[NR];
#pragma unroll
    for (int b = 0; b < NR; ++b) skn[b] = skip_bits(p0, b);
    for (int p = p0; p <= p1; ++p) {
        const bool pv = p <= nz - 2;                          // fine plane p is interior
        const size_t kp = (size_t)p * plane;
        const __amdgpu_buffer_rsrc_t xk = plane_rsrc(x + kp), xn = plane_rsrc(x + (size_t)min(p + 1, nz - 1) * plane);
        const __amdgpu_buffer_rsrc_t rk = plane_rsrc(rho + kp), rik = plane_rsrc(ri + kp);
        V xp[NR], rh[NR], ri4[NR];
        uint32_t sk[NR];
        T lf[NR], p5[NR], q5[NR], h5[NR], ri5[NR];
#pragma unroll
        for (int b = 0; b < NR; ++b) {
            const uint32_t o = ox[b + 1];
            sk[b] = skn[b];
            skn[b] = skip_bits(min(p + 1, nz - 1), b);
            xp[b] = bload4<T>(xn, o);
            rh[b] = bload4<T>(rk, o);
            // the residual at the lane's solid and irregular nodes (issued with the other loads)
            if (sk[b]) ri4[b] = bload4<T>(rik, o);
            else ri4[b] = V{T(0), T(0), T(0), T(0)};
            ri5[b] = (FIFTH && ((sk[b] >> 4) & 1u)) ? bload1<T>(rik, o + 4 * sizeof(T)) : T(0);
            lf[b] = needl ? bload1<T>(xk, o - sizeof(T)) : T(0);
            p5[b] = need5 ? bload1<T>(xn, o + 4 * sizeof(T)) : T(0);
            q5[b] = need5 ? bload1<T>(xk, o + 5 * sizeof(T)) : T(0);
            h5[b] = need5 ? bload1<T>(rk, o + 4 * sizeof(T)) : T(0);
        }
        // the outer y neighbours: x rows 0 and NR + 1
        const V ylo = bload4<T>(xk, ox[0]), yhi = bload4<T>(xk, ox[NR + 1]);
        const T ylo5 = need5 ? bload1<T>(xk, ox[0] + 4 * sizeof(T)) : T(0);
        const T yhi5 = need5 ? bload1<T>(xk, ox[NR + 1] + 4 * sizeof(T)) : T(0);
        const T *cz = cf.c[2] + 8 * p;
        const T za = wave_uniform(cz[5]), zb = wave_uniform(cz[6]), zc = wave_uniform(cz[7]);
        T xr0[NR], xr1[NR];
#pragma unroll
        for (int b = 0; b < NR; ++b) {
            const V &s4 = b == 0 ? ylo : xc[b - 1];
            const V &n4 = b == NR - 1 ? yhi : xc[b + 1];
            const T cv[5] = {xc[b].x, xc[b].y, xc[b].z, xc[b].w, c5[b]};
            const T sv[5] = {s4.x, s4.y, s4.z, s4.w, b == 0 ? ylo5 : c5[b - 1]};
            const T nw[5] = {n4.x, n4.y, n4.z, n4.w, b == NR - 1 ? yhi5 : c5[b + 1]};
            const T mv[5] = {xm[b].x, xm[b].y, xm[b].z, xm[b].w, m5[b]};
            const T uv[5] = {xp[b].x, xp[b].y, xp[b].z, xp[b].w, p5[b]};
            const T rv[5] = {rh[b].x, rh[b].y, rh[b].z, rh[b].w, h5[b]};
            T left = __shfl_up(cv[3], 1, 64), right = __shfl_down(cv[0], 1, 64);
            if (lane == 0) left = lf[b];
            if (lane == 63) right = c5[b];
            // x neighbours of the five nodes: node u's -x one is wxn[u], its +x one exn[u]
            const T wxn[5] = {left, cv[0], cv[1], cv[2], cv[3]};
            const T exn[5] = {cv[1], cv[2], cv[3], right, q5[b]};
            T r[5];
#pragma unroll
            for (int u = 0; u < 5; ++u)
                r[u] = mg_reg_resid(rv[u], cv[u], wxn[u], exn[u], sv[u], nw[u], mv[u], uv[u], kax[u], kbx[u],
                                    kcx[u], kay[b], kby[b], kcy[b], za, zb, zc);
            // solid or irregular nodes: their residual from ri (0 at a solid node)
            const T qv[5] = {ri4[b].x, ri4[b].y, ri4[b].z, ri4[b].w, ri5[b]};
#pragma unroll
            for (int u = 0; u < 5; ++u) r[u] = ((sk[b] >> u) & 1u) ? qv[u] : r[u];
            const bool live = pv && rok[b];
#pragma unroll
            for (int u = 0; u < 4; ++u) r[u] = (live && u < nv) ? r[u] : T(0);
            T v4 = __shfl_down(r[0], 1, 64);
            if (lane == 63) v4 = (live && need5) ? r[4] : T(0);
            xr0[b] = w0[0] * r[0] + w0[1] * r[1] + w0[2] * r[2];
            xr1[b] = w1[0] * r[2] + w1[1] * r[3] + w1[2] * v4;
        }
        if (p & 1) {
            // fine plane 2K + 1: the last of coarse plane K, the first of K + 1
            const int K = (p - 1) >> 1;
            if (K >= K0) {
                add_plane(K, 2, xr0, xr1);
                emit(K);
            }
            if (K + 1 < K1) {
                open(K + 1);
                add_plane(K + 1, 0, xr0, xr1);
            }
        } else {
            add_plane(p >> 1, 1, xr0, xr1);
        }
#pragma unroll
        for (int b = 0; b < NR; ++b) {
            xm[b] = xc[b];
            xc[b] = xp[b];
            m5[b] = c5[b];
            c5[b] = p5[b];
        }
    }
}

// x(i, j, k) += (P e)(i, j, k) at the regular unknown fine nodes; an irregular node (next
// to the body) keeps x and gets its correction from the post-smoothing.  Interpolating the
// coarse correction there, from coarse nodes that see another interface position, makes the
// cycle amplify errors next to the body (a V-cycle with 3 + 3 steps then grows the error
// 7.6-fold per cycle on 64^3 with 8 spheres; without those corrections it contracts by 0.3).
// Block 64 x 4: lane l of
// wavefront w takes the interior nodes i0 .. i0 + 3 (i0 = 1 + 256 blockIdx.x + 4 l) of row
// j = 1 + 4 blockIdx.y + w in the planes k = 2 blockIdx.z and 2 blockIdx.z + 1 (the interior
// ones), which interpolate from the same two coarse planes.  A fine point i lies in the
// coarse interval starting at min(i / 2, nc - 2) (coarse point I is fine point 2I, the last
// one excepted), so the lane's nodes interpolate from the four coarse x points a0 .. a0 + 3
// of four coarse rows.  Every load is issued at once (4-vectors: x of both planes, the four
// coarse rows, the x weights; vectors and weight tables carry padding past their ends): the
// coarse rows are combined in y, then in z for each plane, then each node interpolates in
// x.  x is stored as one 4-vector where all four nodes are unknowns.
template <typename T>
__global__ void __launch_bounds__(256) k_mg_prolong_add(int nfx, int nfy, int nfz, int ncx, int ncy, int ncz,
                                                        MgAxis<T> ax, MgAxis<T> ay, MgAxis<T> az,
                                                        const uint32_t *__restrict__ skip, int W,
                                                        const T *__restrict__ e, T *__restrict__ x)
{
    using V = typename MgVec4<T>::type;
    const int j = 1 + (int)(blockIdx.y * 4 + threadIdx.y), kp = 2 * (int)blockIdx.z;
    const int i0 = 1 + (int)(blockIdx.x * 256 + 4 * threadIdx.x);
    if (j > nfy - 2 || i0 > nfx - 2) return;
    const int nv = min(4, nfx - 1 - i0);
    const int a0 = min(i0 >> 1, ncx - 2), b = min(j >> 1, ncy - 2), c = min(kp >> 1, ncz - 2);
    const size_t cplane = (size_t)ncx * ncy, fplane = (size_t)nfx * nfy;
    const T *e00 = e + (size_t)c * cplane + (size_t)b * ncx + a0;   // coarse (a0, b, c)
    bool ok[2];
    size_t ef[2];
    V xv[2];
    uint32_t sk[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = kp + h;
        ok[h] = k >= 1 && k <= nfz - 2;
        const int kc = ok[h] ? k : 1;
        ef[h] = (size_t)i0 + (size_t)nfx * j + (size_t)kc * fplane;
        xv[h] = *reinterpret_cast<const V *>(x + ef[h]);
        // skip bits (solid and irregular nodes) of nodes i0 .. i0 + 3: words read in pairs,
        // the array carries two words of padding
        const uint32_t *w = skip + ((size_t)kc * nfy + j) * W + (i0 >> 5);
        sk[h] = (uint32_t)((((uint64_t)w[0]) | ((uint64_t)w[1] << 32)) >> (i0 & 31)) & 0xFu;
    }
    const V q00 = *reinterpret_cast<const V *>(e00);
    const V q10 = *reinterpret_cast<const V *>(e00 + ncx);
    const V q01 = *reinterpret_cast<const V *>(e00 + cplane);
    const V q11 = *reinterpret_cast<const V *>(e00 + cplane + ncx);
    const V wxv = *reinterpret_cast<const V *>(ax.pw + i0);
    const T wy = ay.pw[j];
    const V lo = (T(1) - wy) * q00 + wy * q10, hi = (T(1) - wy) * q01 + wy * q11;   // y, coarse planes c, c + 1
    const T wx[4] = {wxv.x, wxv.y, wxv.z, wxv.w};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (!ok[h]) continue;
        const T wz = az.pw[kp + h];
        const V r4 = (T(1) - wz) * lo + wz * hi;
        const T ryz[4] = {r4.x, r4.y, r4.z, r4.w};
        T add[4];
        bool m[4];
        bool all = nv == 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int d = min((i0 + u) >> 1, ncx - 2) - a0;   // 0 .. 2
            const T l = d == 0 ? ryz[0] : (d == 1 ? ryz[1] : ryz[2]);
            const T r = d == 0 ? ryz[1] : (d == 1 ? ryz[2] : ryz[3]);
            add[u] = (T(1) - wx[u]) * l + wx[u] * r;
            m[u] = u < nv && !((sk[h] >> u) & 1u);   // regular unknowns only (interior, no skip bit)
            all = all && m[u];
        }
        V xo = xv[h];
        if (all) {
            xo.x += add[0];
            xo.y += add[1];
            xo.z += add[2];
            xo.w += add[3];
            *reinterpret_cast<V *>(x + ef[h]) = xo;
        } else {
            const T xs[4] = {xo.x, xo.y, xo.z, xo.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (m[u]) x[ef[h] + u] = xs[u] + add[u];
        }
    }
}

// The coarsest level's Chebyshev-Jacobi iteration on K x = rho from x = 0, all `steps` steps
// in one workgroup (the level has at most MG_LDS_NODES interior nodes): x_k lives in LDS
// (interior nodes, x fastest); each thread keeps, for its nodes q = t + MG_LDS_THREADS u,
// x_{k-1} and the K row and rho divided by the row's diagonal (the tables' regular row, or
// the stored Shortley-Weller row of an irregular node) in registers.  x_k and x_{k+1} live
// in two LDS arrays that swap roles every step, one barrier apart.  Wall neighbours hold 0
// in every iterate and get coefficient 0; solid nodes are never written.  x_steps goes to
// the unknown nodes of out.
template <typename T>
__global__ void __launch_bounds__(MG_LDS_THREADS) k_mg_coarsest(int nx, int ny, int nz, Coef<T> cf,
                                                                const int8_t *__restrict__ type,
                                                                const int *__restrict__ irr_map,
                                                                const T *__restrict__ k7, const T *__restrict__ rho,
                                                                T *__restrict__ out, int steps,
                                                                const T *__restrict__ c1, const T *__restrict__ c2,
                                                                const DevState *st)
{
    constexpr int NPT = MG_LDS_NODES / MG_LDS_THREADS;
    __shared__ T xa[MG_LDS_NODES], xb[MG_LDS_NODES];   // x_k and x_{k+1}, swapped every step
    __shared__ T cs[2 * MG_MAX_COARSE_STEPS];
    if (st && st->done) return;
    const int ni = nx - 2, nj = ny - 2, nk = nz - 2, nij = ni * nj, nint = nij * nk;
    const int t = (int)threadIdx.x;
    if (t < steps) {
        cs[t] = c1[t];
        cs[MG_MAX_COARSE_STEPS + t] = c2[t];
    }
    T kd[NPT], ko[NPT][6], rh[NPT], xp[NPT];
    unsigned inm[NPT];                 // bit v: neighbour v (-x, +x, -y, +y, -z, +z) is interior
    bool act[NPT];
    auto node_of = [&](int q) {
        const int i = 1 + q % ni, j = 1 + (q / ni) % nj, k = 1 + q / nij;
        return (size_t)i + (size_t)nx * (j + (size_t)ny * k);
    };
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int q = t + MG_LDS_THREADS * u;
        xa[q] = T(0);
        xb[q] = T(0);
        xp[u] = T(0);
        act[u] = false;
        kd[u] = T(1);
        rh[u] = T(0);
        inm[u] = 0u;
#pragma unroll
        for (int v = 0; v < 6; ++v) ko[u][v] = T(0);
        // the loads that do not depend on the node's type are issued at once (a point past
        // the level's interior reads node 0), so only an irregular row's stored K row waits
        // for a first round trip
        const bool in = q < nint;
        const int qq = in ? q : 0;
        const int i = 1 + qq % ni, j = 1 + (qq / ni) % nj, k = 1 + qq / nij;
        const size_t e = in ? node_of(q) : 0;
        const int8_t ty_l = type[e];
        const T r_l = rho[e];
        const int ir_l = irr_map[e];
        const T *cx = cf.c[0] + 8 * i, *cy = cf.c[1] + 8 * j, *cz = cf.c[2] + 8 * k;
        const T cx5 = cx[5], cx6 = cx[6], cx7 = cx[7], cy5 = cy[5], cy6 = cy[6], cy7 = cy[7];
        const T cz5 = cz[5], cz6 = cz[6], cz7 = cz[7];
        const int8_t ty = in ? ty_l : (int8_t)0;
        act[u] = ty == 1 || ty == 2;
        if (!act[u]) continue;
        rh[u] = r_l;
        if (ty == 2) {
            const T *row = k7 + 7 * (size_t)ir_l;
            kd[u] = row[0];
#pragma unroll
            for (int v = 0; v < 6; ++v) ko[u][v] = row[1 + v];
        } else {
            kd[u] = cx6 + cy6 + cz6;
            ko[u][0] = cx5; ko[u][1] = cx7;
            ko[u][2] = cy5; ko[u][3] = cy7;
            ko[u][4] = cz5; ko[u][5] = cz7;
        }
        // a wall neighbour is read as the node itself with coefficient 0
        inm[u] = (i > 1 ? 1u : 0u) | (i < nx - 2 ? 2u : 0u) | (j > 1 ? 4u : 0u) | (j < ny - 2 ? 8u : 0u) |
                 (k > 1 ? 16u : 0u) | (k < nz - 2 ? 32u : 0u);
#pragma unroll
        for (int v = 0; v < 6; ++v)
            if (!((inm[u] >> v) & 1u)) ko[u][v] = T(0);
    }
    // rows scaled by 1 / diag K: (rho - K x) / diag = rho' - x - sum_v ko'_v x_v
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const T rd = T(1) / kd[u];
        rh[u] *= rd;
#pragma unroll
        for (int v = 0; v < 6; ++v) ko[u][v] *= rd;
    }
    __syncthreads();
    const int d[6] = {-1, 1, -ni, ni, -nij, nij};
    // step s reads x_s from one array and writes x_{s+1} into the other (nodes that are not
    // unknowns stay 0 in both), so one barrier per step separates them
    T *cur = xa, *nxt = xb;
    for (int s = 0; s < steps; ++s) {
        const T a1 = cs[s], a2 = cs[MG_MAX_COARSE_STEPS + s];
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int q = t + MG_LDS_THREADS * u;
            const T x0 = cur[q];
            T kx = x0;
#pragma unroll
            for (int v = 0; v < 6; ++v) kx += ko[u][v] * cur[((inm[u] >> v) & 1u) ? q + d[v] : q];
            if (act[u]) nxt[q] = x0 + a1 * (x0 - xp[u]) + a2 * (rh[u] - kx);
            xp[u] = x0;
        }
        __syncthreads();
        T *const tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
#pragma unroll
    for (int u = 0; u < NPT; ++u)
        if (act[u]) out[node_of(t + MG_LDS_THREADS * u)] = cur[t + MG_LDS_THREADS * u];
}

// Temporally blocked Chebyshev-Jacobi steps on a coarse level (launch_mg_smooth_tb).  The
// block's extended tile has E = MG_TB_TS + 2 MG_TB_H nodes per direction starting at node
// 1 + MG_TB_TS blockIdx - MG_TB_H; point q = t + MG_TB_THREADS u of it (x fastest) belongs to
// thread t.  x_k of the extended tile lives in LDS (0 at nodes that are not unknowns and at
// nodes outside the grid's interior); each thread keeps x_{k-1}, rho and the K row of its
// points in registers (the regular rows' from the 1D tables, an irregular row's stored
// Shortley-Weller row).  A neighbour outside the extended tile reads 0: that error enters the
// outermost layer at the first step and moves in one layer per step, so after s <= MG_TB_H
// steps the tile (and, for s < MG_TB_H, its first neighbour layer, which the residual reads)
// holds exactly the values of s single sweeps.  The arithmetic is that of the single sweep
// (k_cheb4m): K x = diag x + the six neighbour terms, x_{k+1} = x_k + c1 (x_k - x_{k-1}) +
// c2 (rho - K x) / diag.  The levels this runs on are small enough that a sweep is bound by
// its launch and latency, not by bandwidth: the redundant work on the layers around the tile
// costs less than the launches it saves.
constexpr int MG_TB_E = MG_TB_TS + 2 * MG_TB_H;
constexpr int MG_TB_E3 = MG_TB_E * MG_TB_E * MG_TB_E;
constexpr int MG_TB_NPT = (MG_TB_E3 + MG_TB_THREADS - 1) / MG_TB_THREADS;

// What a temporally blocked pass writes besides x on its tile: nothing (TB_X), the residual
// on the tile (TB_RES), or the residual restricted into the next coarser level (TB_RESTRICT:
// that level's rho and first step, as k_mg_restrict forms them, for the coarse nodes whose
// centre lies in the tile; the residual is formed on the tile and one layer around it, which
// needs the pass to leave two layers exact, S.n <= MG_TB_H - 2).  With PRO the pass starts
// from x + P e at the regular unknowns (the coarse correction added on load, as
// k_mg_prolong_add forms it) instead of x.
enum { TB_X = 0, TB_RES = 1, TB_RESTRICT = 2 };

template <typename T, int OUT, bool PRO>
__global__ void __launch_bounds__(MG_TB_THREADS, sizeof(T) == 4 ? 8 : 1) k_mg_smooth_tb(int nx, int ny, int nz, Coef<T> cf,
                                                                const int8_t *__restrict__ type,
                                                                const int *__restrict__ irr_map,
                                                                const T *__restrict__ k7, const T *__restrict__ rho,
                                                                const T *__restrict__ xin, T *__restrict__ xout,
                                                                T *__restrict__ rout, MgSteps<T> S, const DevState *st,
                                                                MgTransfer<T> tr, const T *__restrict__ ec,
                                                                T *__restrict__ rc, MgFirst<T> F)
{
    constexpr int E = MG_TB_E, E2 = E * E, NPT = MG_TB_NPT;
    static_assert(MG_TB_TS % 2 == 0, "a tile holds whole coarse cells");
    __shared__ T xs[MG_TB_E3];
    __shared__ T rs[OUT == TB_RESTRICT ? MG_TB_E3 : 1];
    if (st && st->done) return;
    const int t = (int)threadIdx.x;
    const int o[3] = {1 + MG_TB_TS * (int)blockIdx.x - MG_TB_H, 1 + MG_TB_TS * (int)blockIdx.y - MG_TB_H,
                      1 + MG_TB_TS * (int)blockIdx.z - MG_TB_H};
    T xp[NPT], rh[NPT], kd[NPT], ko[NPT][6];
    bool act[NPT];
    // TB_RESTRICT: thread t < (TS/2)^3 restricts into coarse node (I, J, K) = (1 + TS/2 b + c)
    // at the end; its nine weights and the node's diagonal are loaded with the tile and kept
    // in LDS until then
    constexpr int CT = MG_TB_TS / 2, CT3 = CT * CT * CT;
    __shared__ T rsw[OUT == TB_RESTRICT ? CT3 : 1][10];
    const int ci = t % CT, cj = (t / CT) % CT, ck = t / (CT * CT);
    const int cI = 1 + CT * (int)blockIdx.x + ci, cJ = 1 + CT * (int)blockIdx.y + cj, cK = 1 + CT * (int)blockIdx.z + ck;
    const bool cown = OUT == TB_RESTRICT && t < CT3 && cI <= tr.nc[0] - 2 && cJ <= tr.nc[1] - 2 && cK <= tr.nc[2] - 2;
    const size_t ce = cown ? (size_t)cI + (size_t)tr.nc[0] * (cJ + (size_t)tr.nc[1] * cK) : 0;
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int q = t + MG_TB_THREADS * u;
        const int ii = q % E, jj = (q / E) % E, kk = q / E2;
        const int i = o[0] + ii, j = o[1] + jj, k = o[2] + kk;
        const bool in = q < MG_TB_E3 && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2;
        const size_t e = in ? (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k) : 0;
        // every load that does not depend on the node's type is issued at once (e and the
        // clamped indices address valid entries for any point), so only an irregular row's
        // stored K row waits for a first round trip
        const int ic = min(max(i, 1), nx - 2), jc = min(max(j, 1), ny - 2), kc = min(max(k, 1), nz - 2);
        const int8_t ty_l = type[e];
        const T x_l = xin[e], r_l = rho[e];
        const int ir_l = irr_map[e];
        const T *cx = cf.c[0] + 8 * ic, *cy = cf.c[1] + 8 * jc, *cz = cf.c[2] + 8 * kc;
        const T cx5 = cx[5], cx6 = cx[6], cx7 = cx[7], cy5 = cy[5], cy6 = cy[6], cy7 = cy[7];
        const T cz5 = cz[5], cz6 = cz[6], cz7 = cz[7];
        const int8_t ty = in ? ty_l : (int8_t)0;
        act[u] = ty == 1 || ty == 2;
        T x0 = act[u] ? x_l : T(0);
        if (PRO) {
            // (P e)(i, j, k): the coarse interval of each index, combined in y, then z, then x
            const int ncx = tr.nc[0], ncy = tr.nc[1], ncz = tr.nc[2];
            const int a0 = min(ic >> 1, ncx - 2), b0 = min(jc >> 1, ncy - 2), c0 = min(kc >> 1, ncz - 2);
            const size_t cpl = (size_t)ncx * ncy;
            const T *e00 = ec + (size_t)c0 * cpl + (size_t)b0 * ncx + a0;
            const T wx = tr.ax[0].pw[ic], wy = tr.ax[1].pw[jc], wz = tr.ax[2].pw[kc];
            T ryz[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const T lo = (T(1) - wy) * e00[h] + wy * e00[ncx + h];
                const T hi = (T(1) - wy) * e00[cpl + h] + wy * e00[cpl + ncx + h];
                ryz[h] = (T(1) - wz) * lo + wz * hi;
            }
            const T add = (T(1) - wx) * ryz[0] + wx * ryz[1];
            if (ty == 1) x0 = x0 + add;
        }
        if (q < MG_TB_E3) xs[q] = x0;
        rh[u] = act[u] ? r_l : T(0);
        xp[u] = T(0);
        kd[u] = T(1);
#pragma unroll
        for (int v = 0; v < 6; ++v) ko[u][v] = T(0);
        if (ty == 2) {
            const T *r = k7 + 7 * (size_t)ir_l;
            kd[u] = r[0];
#pragma unroll
            for (int v = 0; v < 6; ++v) ko[u][v] = r[1 + v];
        } else if (ty == 1) {
            kd[u] = (cx6 + cy6) + cz6;
            ko[u][0] = cx5; ko[u][1] = cx7;
            ko[u][2] = cy5; ko[u][3] = cy7;
            ko[u][4] = cz5; ko[u][5] = cz7;
        }
    }
    if (cown) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            rsw[t][c] = tr.ax[0].rw[3 * cI + c];
            rsw[t][3 + c] = tr.ax[1].rw[3 * cJ + c];
            rsw[t][6 + c] = tr.ax[2].rw[3 * cK + c];
        }
        rsw[t][9] = F.diag[ce];
    }
    __syncthreads();
    // K x at point q of the LDS tile (neighbours outside the extended tile read 0)
    auto kx_of = [&](int u, int q, T x0) {
        const int ii = q % E, jj = (q / E) % E, kk = q / E2;
        const T w = ii > 0 ? xs[q - 1] : T(0), ea = ii < E - 1 ? xs[q + 1] : T(0);
        const T sv = jj > 0 ? xs[q - E] : T(0), nv = jj < E - 1 ? xs[q + E] : T(0);
        const T mv = kk > 0 ? xs[q - E2] : T(0), uv = kk < E - 1 ? xs[q + E2] : T(0);
        return kd[u] * x0 + ko[u][0] * w + ko[u][1] * ea + ko[u][2] * sv + ko[u][3] * nv + ko[u][4] * mv +
               ko[u][5] * uv;
    };
    for (int s = 0; s < S.n; ++s) {
        const T c1 = S.c1[s], c2 = S.c2[s];
        T xn[NPT];
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int q = t + MG_TB_THREADS * u;
            xn[u] = T(0);
            if (!act[u]) continue;
            const T x0 = xs[q];
            const T kx = kx_of(u, q, x0);
            xn[u] = x0 + c1 * (x0 - xp[u]) + c2 * (rh[u] - kx) / kd[u];
            xp[u] = x0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NPT; ++u)
            if (act[u]) xs[t + MG_TB_THREADS * u] = xn[u];
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int q = t + MG_TB_THREADS * u;
        const int ii = q % E, jj = (q / E) % E, kk = q / E2;
        if (OUT == TB_RESTRICT && q < MG_TB_E3) {
            // the residual on the tile and the layer around it, 0 elsewhere and off the unknowns
            const bool near = ii >= MG_TB_H - 1 && ii <= MG_TB_H + MG_TB_TS && jj >= MG_TB_H - 1 &&
                              jj <= MG_TB_H + MG_TB_TS && kk >= MG_TB_H - 1 && kk <= MG_TB_H + MG_TB_TS;
            rs[q] = (act[u] && near) ? rh[u] - kx_of(u, q, xs[q]) : T(0);
        }
        if (!act[u] || ii < MG_TB_H || ii >= MG_TB_H + MG_TB_TS || jj < MG_TB_H || jj >= MG_TB_H + MG_TB_TS ||
            kk < MG_TB_H || kk >= MG_TB_H + MG_TB_TS)
            continue;
        const size_t e = (size_t)(o[0] + ii) + (size_t)nx * ((size_t)(o[1] + jj) + (size_t)ny * (o[2] + kk));
        const T x0 = xs[q];
        xout[e] = x0;
        if (OUT == TB_RES) rout[e] = rh[u] - kx_of(u, q, x0);
    }
    if (OUT == TB_RESTRICT) {
        // coarse node (I, J, K): its fine points 2I - 1 .. 2I + 1 are the extended-tile points
        // H + 2c .. H + 2c + 2 of each direction
        __syncthreads();
        if (cown) {
            const int i0 = MG_TB_H + 2 * ci, j0 = MG_TB_H + 2 * cj, k0 = MG_TB_H + 2 * ck;
            const T *w = rsw[t];
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const T wyz = w[6 + c] * w[3 + b];
                    const T *row = rs + (k0 + c) * E2 + (j0 + b) * E + i0;
                    acc += wyz * (w[0] * row[0] + w[1] * row[1] + w[2] * row[2]);
                }
            }
            const T cdg = w[9];
            rc[ce] = cdg != T(0) ? acc : T(0);
            if (F.x1 && cdg != T(0)) F.x1[ce] = F.c2 * acc / cdg;
        }
    }
}

// diag[e] = the diagonal of K at node e if it is an unknown (the 1D tables of a regular node,
// summed as cx + (cy + cz), or the stored row of an irregular one), 0 otherwise
template <typename T>
__global__ void k_mg_diag(int nx, int ny, int nz, Coef<T> cf, const int8_t *__restrict__ type,
                          const int *__restrict__ irr_map, const T *__restrict__ k7, T *__restrict__ diag)
{
    const size_t n = (size_t)nx * ny * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((size_t)nx * ny));
        const int8_t t = type[e];
        T d = T(0);
        if (t == 1) d = cf.c[0][8 * i + 6] + (cf.c[1][8 * j + 6] + cf.c[2][8 * k + 6]);
        else if (t == 2) d = k7[7 * (size_t)irr_map[e]];
        diag[e] = d;
    }
}

// map[node] = irregular row of the node (the rows list nodes in increasing order)
__global__ void k_mg_irr_map(int nirr, const int *__restrict__ nodes, int *__restrict__ map)
{
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r < nirr) map[nodes[r]] = r;
}

}  // namespace

template <typename T>
void launch_mg_diag(hipStream_t s, int nx, int ny, int nz, const Coef<T> &cf, const int8_t *type, const int *irr_map,
                    const T *k7, T *diag)
{
    const size_t n = (size_t)nx * ny * nz;
    k_mg_diag<T><<<(unsigned)std::min<size_t>((n + 255) / 256, 4096), 256, 0, s>>>(nx, ny, nz, cf, type, irr_map, k7,
                                                                                  diag);
}

template <typename T>
void launch_mg_restrict(hipStream_t s, const MgTransfer<T> &t, const T *r, T *rc, const MgFirst<T> &first)
{
    dim3 grid((unsigned)((t.nc[0] - 2 + 127) / 128), (unsigned)((t.nc[1] - 2 + 3) / 4), (unsigned)(t.nc[2] - 2));
    k_mg_restrict<T><<<grid, dim3(64, 4), 0, s>>>(t.nc[0], t.nc[1], t.nf[0], t.nf[1], t.ax[0], t.ax[1], t.ax[2], r,
                                                  rc, first);
}

// coarse rows per wavefront of the fused residual and restriction
constexpr int RR_ROWS = 1;

template <typename T>
void launch_mg_resid_restrict(hipStream_t s, const Geom &g, const Coef<T> &cf, const uint32_t *skip, const T *x,
                              const T *rho, const T *ri, const MgTransfer<T> &t, T *rc, const MgFirst<T> &first,
                              const DevState *st)
{
    // the fifth-node path (more registers) only where a further segment exists
    const int ncx = t.nc[0], ncy = t.nc[1], ncz = t.nc[2];
    const bool fifth = (ncx - 2 + 127) / 128 > 1;
    const void *fn = fifth ? reinterpret_cast<const void *>(&k_mg_resid_restrict<T, true, RR_ROWS>)
                           : reinterpret_cast<const void *>(&k_mg_resid_restrict<T, false, RR_ROWS>);
    // The march is bound by the latency of its plane steps: all blocks run in one round,
    // as many as fit on the device at once (z-chunks of at least two coarse planes).
    static int per_cu[2] = {0, 0};
    if (!per_cu[fifth]) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0) != hipSuccess || nb < 1) nb = 1;
        per_cu[fifth] = nb;
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    Tiling tl{};
    tl.tw = 128;
    tl.ty = 4 * RR_ROWS;
    tl.tiles_x = (ncx - 2 + 127) / 128;
    tl.tiles_y = (ncy - 2 + tl.ty - 1) / tl.ty;
    const int nzi = ncz - 2, per_plane = tl.tiles_x * tl.tiles_y;
    const int want = std::max(1, per_cu[fifth] * ncu / per_plane);
    tl.TZ = std::max(std::min(2, nzi), (nzi + want - 1) / want);
    tl.zchunks = (nzi + tl.TZ - 1) / tl.TZ;
    tl.ntiles = per_plane * tl.zchunks;
    tl.nblk = (tl.ntiles + NXCD - 1) / NXCD * NXCD;
    if (fifth)
        k_mg_resid_restrict<T, true, RR_ROWS><<<tl.nblk, dim3(64, 4), 0, s>>>(
            g, tl, cf, skip, x, rho, ri, ncx, ncy, ncz, t.ax[0], t.ax[1], t.ax[2], rc, first, st);
    else
        k_mg_resid_restrict<T, false, RR_ROWS><<<tl.nblk, dim3(64, 4), 0, s>>>(
            g, tl, cf, skip, x, rho, ri, ncx, ncy, ncz, t.ax[0], t.ax[1], t.ax[2], rc, first, st);
}

template <typename T>
void launch_mg_prolong_add(hipStream_t s, const MgTransfer<T> &t, const uint32_t *skip_f, int W, const T *e, T *x)
{
    // blockIdx.z = p covers fine planes 2p and 2p + 1 (interior planes 1 .. nf[2] - 2)
    dim3 grid((unsigned)((t.nf[0] - 2 + 255) / 256), (unsigned)((t.nf[1] - 2 + 3) / 4), (unsigned)((t.nf[2] - 2) / 2 + 1));
    k_mg_prolong_add<T><<<grid, dim3(64, 4), 0, s>>>(t.nf[0], t.nf[1], t.nf[2], t.nc[0], t.nc[1], t.nc[2], t.ax[0],
                                                     t.ax[1], t.ax[2], skip_f, W, e, x);
}

template <typename T>
void launch_mg_coarsest(hipStream_t s, int nx, int ny, int nz, const Coef<T> &cf, const int8_t *type,
                        const int *irr_map, const T *k7, const T *rho, T *out, int steps, const T *c1, const T *c2,
                        const DevState *st)
{
    k_mg_coarsest<T><<<1, MG_LDS_THREADS, 0, s>>>(nx, ny, nz, cf, type, irr_map, k7, rho, out, steps, c1, c2, st);
}

template <typename T>
void launch_mg_smooth_tb(hipStream_t s, int nx, int ny, int nz, const Coef<T> &cf, const int8_t *type,
                         const int *irr_map, const T *k7, const T *rho, const T *xin, T *xout, T *rout,
                         const MgSteps<T> &S, const DevState *st, const MgTransfer<T> *tr, const T *e_add, T *rc,
                         const MgFirst<T> *first)
{
    const dim3 grid((unsigned)((nx - 2 + MG_TB_TS - 1) / MG_TB_TS), (unsigned)((ny - 2 + MG_TB_TS - 1) / MG_TB_TS),
                    (unsigned)((nz - 2 + MG_TB_TS - 1) / MG_TB_TS));
    const MgTransfer<T> t = tr ? *tr : MgTransfer<T>{};
    const MgFirst<T> F = first ? *first : MgFirst<T>{};
#define CPS_TB_LAUNCH(OUT, PRO)                                                                                        \
    k_mg_smooth_tb<T, OUT, PRO><<<grid, MG_TB_THREADS, 0, s>>>(nx, ny, nz, cf, type, irr_map, k7, rho, xin, xout, rout, \
                                                               S, st, t, e_add, rc, F)
    if (rc) CPS_TB_LAUNCH(TB_RESTRICT, false);
    else if (rout) CPS_TB_LAUNCH(TB_RES, false);
    else if (e_add) CPS_TB_LAUNCH(TB_X, true);
    else CPS_TB_LAUNCH(TB_X, false);
#undef CPS_TB_LAUNCH
}

void launch_mg_irr_map(hipStream_t s, int nirr, const int *nodes, int *map)
{
    if (nirr > 0) k_mg_irr_map<<<(nirr + 255) / 256, 256, 0, s>>>(nirr, nodes, map);
}

template void launch_mg_coarsest<double>(hipStream_t, int, int, int, const Coef<double> &, const int8_t *, const int *,
                                         const double *, const double *, double *, int, const double *, const double *,
                                         const DevState *);
template void launch_mg_coarsest<float>(hipStream_t, int, int, int, const Coef<float> &, const int8_t *, const int *,
                                        const float *, const float *, float *, int, const float *, const float *,
                                        const DevState *);
template void launch_mg_smooth_tb<double>(hipStream_t, int, int, int, const Coef<double> &, const int8_t *,
                                          const int *, const double *, const double *, const double *, double *,
                                          double *, const MgSteps<double> &, const DevState *,
                                          const MgTransfer<double> *, const double *, double *,
                                          const MgFirst<double> *);
template void launch_mg_smooth_tb<float>(hipStream_t, int, int, int, const Coef<float> &, const int8_t *, const int *,
                                         const float *, const float *, const float *, float *, float *,
                                         const MgSteps<float> &, const DevState *, const MgTransfer<float> *,
                                         const float *, float *, const MgFirst<float> *);
template void launch_mg_restrict<double>(hipStream_t, const MgTransfer<double> &, const double *, double *,
                                         const MgFirst<double> &);
template void launch_mg_restrict<float>(hipStream_t, const MgTransfer<float> &, const float *, float *,
                                        const MgFirst<float> &);
template void launch_mg_diag<double>(hipStream_t, int, int, int, const Coef<double> &, const int8_t *, const int *,
                                     const double *, double *);
template void launch_mg_diag<float>(hipStream_t, int, int, int, const Coef<float> &, const int8_t *, const int *,
                                    const float *, float *);
template void launch_mg_resid_restrict<double>(hipStream_t, const Geom &, const Coef<double> &, const uint32_t *, const double *, const double *,
                                                const double *, const MgTransfer<double> &, double *,
                                                const MgFirst<double> &, const DevState *);
template void launch_mg_resid_restrict<float>(hipStream_t, const Geom &, const Coef<float> &, const uint32_t *, const float *, const float *,
                                               const float *, const MgTransfer<float> &, float *,
                                               const MgFirst<float> &, const DevState *);
template void launch_mg_prolong_add<double>(hipStream_t, const MgTransfer<double> &, const uint32_t *, int,
                                            const double *, double *);
template void launch_mg_prolong_add<float>(hipStream_t, const MgTransfer<float> &, const uint32_t *, int, const float *,
                                           float *);

}  // namespace cps
