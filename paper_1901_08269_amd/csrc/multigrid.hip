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
// step from zero, x1 = c2 rho / diag K, at its unknown nodes (the diagonal from the 1D
// tables, or the stored row of an irregular node).
template <typename T>
__global__ void __launch_bounds__(256) k_mg_restrict(int ncx, int ncy, int nfx, int nfy, MgAxis<T> ax, MgAxis<T> ay,
                                                     MgAxis<T> az, const int8_t *__restrict__ type_c,
                                                     const T *__restrict__ r, T *__restrict__ rc, MgFirst<T> F)
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
    const bool unk0 = unknown(type_c[ec]), unk1 = two && unknown(type_c[ec + 1]);
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
        const T dyz = F.cf.c[1][8 * J + 6] + F.cf.c[2][8 * K + 6];
        if (unk0) {
            const T dg = type_c[ec] == 2 ? F.k7[7 * (size_t)F.irr_map[ec]] : F.cf.c[0][8 * I0 + 6] + dyz;
            F.x1[ec] = F.c2 * acc0 / dg;
        }
        if (unk1) {
            const T dg = type_c[ec + 1] == 2 ? F.k7[7 * (size_t)F.irr_map[ec + 1]] : F.cf.c[0][8 * (I0 + 1) + 6] + dyz;
            F.x1[ec + 1] = F.c2 * acc1 / dg;
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
                                                        const int8_t *__restrict__ type_f, const T *__restrict__ e,
                                                        T *__restrict__ x)
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
    int8_t ty[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = kp + h;
        ok[h] = k >= 1 && k <= nfz - 2;
        ef[h] = (size_t)i0 + (size_t)nfx * j + (size_t)(ok[h] ? k : 1) * fplane;
        xv[h] = *reinterpret_cast<const V *>(x + ef[h]);
#pragma unroll
        for (int u = 0; u < 4; ++u) ty[h][u] = type_f[ef[h] + min(u, nv - 1)];
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
            m[u] = u < nv && ty[h][u] == 1;   // regular unknowns only
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
// the stored Shortley-Weller row of an irregular node) in registers.  A barrier separates the reads of x_k from the writes of
// x_{k+1}.  Wall neighbours hold 0 in every iterate and get coefficient 0; solid nodes are
// never written.  x_steps goes to the unknown nodes of out.
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
    __shared__ T xs[MG_LDS_NODES];
    if (st && st->done) return;
    const int ni = nx - 2, nj = ny - 2, nk = nz - 2, nij = ni * nj, nint = nij * nk;
    const int t = (int)threadIdx.x;
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
        xs[q] = T(0);
        xp[u] = T(0);
        act[u] = false;
        kd[u] = T(1);
        rh[u] = T(0);
        inm[u] = 0u;
#pragma unroll
        for (int v = 0; v < 6; ++v) ko[u][v] = T(0);
        if (q >= nint) continue;
        const int i = 1 + q % ni, j = 1 + (q / ni) % nj, k = 1 + q / nij;
        const size_t e = node_of(q);
        const int8_t ty = type[e];
        act[u] = ty == 1 || ty == 2;
        if (!act[u]) continue;
        rh[u] = rho[e];
        if (ty == 2) {
            const T *row = k7 + 7 * (size_t)irr_map[e];
            kd[u] = row[0];
#pragma unroll
            for (int v = 0; v < 6; ++v) ko[u][v] = row[1 + v];
        } else {
            const T *cx = cf.c[0] + 8 * i, *cy = cf.c[1] + 8 * j, *cz = cf.c[2] + 8 * k;
            kd[u] = cx[6] + cy[6] + cz[6];
            ko[u][0] = cx[5]; ko[u][1] = cx[7];
            ko[u][2] = cy[5]; ko[u][3] = cy[7];
            ko[u][4] = cz[5]; ko[u][5] = cz[7];
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
    for (int s = 0; s < steps; ++s) {
        const T a1 = c1[s], a2 = c2[s];
        T xn[NPT];
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int q = t + MG_LDS_THREADS * u;
            const T x0 = xs[q];
            T kx = x0;
#pragma unroll
            for (int v = 0; v < 6; ++v) kx += ko[u][v] * xs[((inm[u] >> v) & 1u) ? q + d[v] : q];
            xn[u] = x0 + a1 * (x0 - xp[u]) + a2 * (rh[u] - kx);
            xp[u] = x0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NPT; ++u)
            if (act[u]) xs[t + MG_LDS_THREADS * u] = xn[u];
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NPT; ++u)
        if (act[u]) out[node_of(t + MG_LDS_THREADS * u)] = xs[t + MG_LDS_THREADS * u];
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

template <typename T, bool RES>
__global__ void __launch_bounds__(MG_TB_THREADS) k_mg_smooth_tb(int nx, int ny, int nz, Coef<T> cf,
                                                                const int8_t *__restrict__ type,
                                                                const int *__restrict__ irr_map,
                                                                const T *__restrict__ k7, const T *__restrict__ rho,
                                                                const T *__restrict__ xin, T *__restrict__ xout,
                                                                T *__restrict__ rout, MgSteps<T> S, const DevState *st)
{
    constexpr int E = MG_TB_E, E2 = E * E, NPT = MG_TB_NPT;
    __shared__ T xs[MG_TB_E3];
    if (st && st->done) return;
    const int t = (int)threadIdx.x;
    const int o[3] = {1 + MG_TB_TS * (int)blockIdx.x - MG_TB_H, 1 + MG_TB_TS * (int)blockIdx.y - MG_TB_H,
                      1 + MG_TB_TS * (int)blockIdx.z - MG_TB_H};
    T xp[NPT], rh[NPT], kd[NPT], ko[NPT][6];
    bool act[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int q = t + MG_TB_THREADS * u;
        const int ii = q % E, jj = (q / E) % E, kk = q / E2;
        const int i = o[0] + ii, j = o[1] + jj, k = o[2] + kk;
        const bool in = q < MG_TB_E3 && i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2 && k >= 1 && k <= nz - 2;
        const size_t e = in ? (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k) : 0;
        const int8_t ty = in ? type[e] : (int8_t)0;
        act[u] = ty == 1 || ty == 2;
        if (q < MG_TB_E3) xs[q] = act[u] ? xin[e] : T(0);
        rh[u] = act[u] ? rho[e] : T(0);
        xp[u] = T(0);
        kd[u] = T(1);
#pragma unroll
        for (int v = 0; v < 6; ++v) ko[u][v] = T(0);
        if (ty == 2) {
            const T *r = k7 + 7 * (size_t)irr_map[e];
            kd[u] = r[0];
#pragma unroll
            for (int v = 0; v < 6; ++v) ko[u][v] = r[1 + v];
        } else if (ty == 1) {
            const T *cx = cf.c[0] + 8 * i, *cy = cf.c[1] + 8 * j, *cz = cf.c[2] + 8 * k;
            kd[u] = (cx[6] + cy[6]) + cz[6];
            ko[u][0] = cx[5]; ko[u][1] = cx[7];
            ko[u][2] = cy[5]; ko[u][3] = cy[7];
            ko[u][4] = cz[5]; ko[u][5] = cz[7];
        }
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
        if (!act[u] || ii < MG_TB_H || ii >= MG_TB_H + MG_TB_TS || jj < MG_TB_H || jj >= MG_TB_H + MG_TB_TS ||
            kk < MG_TB_H || kk >= MG_TB_H + MG_TB_TS)
            continue;
        const size_t e = (size_t)(o[0] + ii) + (size_t)nx * ((size_t)(o[1] + jj) + (size_t)ny * (o[2] + kk));
        const T x0 = xs[q];
        xout[e] = x0;
        if (RES) rout[e] = rh[u] - kx_of(u, q, x0);
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
void launch_mg_restrict(hipStream_t s, const MgTransfer<T> &t, const int8_t *type_c, const T *r, T *rc,
                        const MgFirst<T> &first)
{
    dim3 grid((unsigned)((t.nc[0] - 2 + 127) / 128), (unsigned)((t.nc[1] - 2 + 3) / 4), (unsigned)(t.nc[2] - 2));
    k_mg_restrict<T><<<grid, dim3(64, 4), 0, s>>>(t.nc[0], t.nc[1], t.nf[0], t.nf[1], t.ax[0], t.ax[1], t.ax[2], type_c,
                                                  r, rc, first);
}

template <typename T>
void launch_mg_prolong_add(hipStream_t s, const MgTransfer<T> &t, const int8_t *type_f, const T *e, T *x)
{
    // blockIdx.z = p covers fine planes 2p and 2p + 1 (interior planes 1 .. nf[2] - 2)
    dim3 grid((unsigned)((t.nf[0] - 2 + 255) / 256), (unsigned)((t.nf[1] - 2 + 3) / 4), (unsigned)((t.nf[2] - 2) / 2 + 1));
    k_mg_prolong_add<T><<<grid, dim3(64, 4), 0, s>>>(t.nf[0], t.nf[1], t.nf[2], t.nc[0], t.nc[1], t.nc[2], t.ax[0],
                                                     t.ax[1], t.ax[2], type_f, e, x);
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
                         const MgSteps<T> &S, const DevState *st)
{
    const dim3 grid((unsigned)((nx - 2 + MG_TB_TS - 1) / MG_TB_TS), (unsigned)((ny - 2 + MG_TB_TS - 1) / MG_TB_TS),
                    (unsigned)((nz - 2 + MG_TB_TS - 1) / MG_TB_TS));
    if (rout)
        k_mg_smooth_tb<T, true><<<grid, MG_TB_THREADS, 0, s>>>(nx, ny, nz, cf, type, irr_map, k7, rho, xin, xout, rout,
                                                               S, st);
    else
        k_mg_smooth_tb<T, false><<<grid, MG_TB_THREADS, 0, s>>>(nx, ny, nz, cf, type, irr_map, k7, rho, xin, xout,
                                                                nullptr, S, st);
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
                                          double *, const MgSteps<double> &, const DevState *);
template void launch_mg_smooth_tb<float>(hipStream_t, int, int, int, const Coef<float> &, const int8_t *, const int *,
                                         const float *, const float *, const float *, float *, float *,
                                         const MgSteps<float> &, const DevState *);
template void launch_mg_restrict<double>(hipStream_t, const MgTransfer<double> &, const int8_t *, const double *,
                                         double *, const MgFirst<double> &);
template void launch_mg_restrict<float>(hipStream_t, const MgTransfer<float> &, const int8_t *, const float *, float *,
                                        const MgFirst<float> &);
template void launch_mg_prolong_add<double>(hipStream_t, const MgTransfer<double> &, const int8_t *, const double *,
                                            double *);
template void launch_mg_prolong_add<float>(hipStream_t, const MgTransfer<float> &, const int8_t *, const float *,
                                           float *);

}  // namespace cps
