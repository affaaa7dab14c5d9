// sweeps.hip -- the hot path of the solve: the matrix-free compact operator B (regular rows
// in tiles, irregular rows from their table in the same launch), the Chebyshev-Jacobi
// sweeps of the preconditioner K, and the BiCGSTAB vector updates with their dot products
// reduced in the same launch (Alg. 1 with the split of Eq. Bdec).
//
// Launch shape: the stencil and update kernels run on vectorised rows -- a wavefront owns a
// 256-node segment of an x-row, four nodes per lane -- in blocks of four wavefronts that
// march over z-chunks of the interior (XCD-aware tile order); blocks before (or, for the B
// apply, after) the tiles process the irregular rows; the restart kernel strides over all
// nodes with 16-byte vectors.  Kernels that reduce write one partial per block; a one-block finalize
// kernel that follows sums them in a fixed order (deterministic) and updates the
// device-resident BiCGSTAB scalars, so the host never waits inside an iteration.
#include <hip/hip_ext.h>

#include "cps_device.h"
#include "cps_kernels.h"

namespace cps {

// Blocks that process irregular rows come in a count rounded up to a multiple of the XCD
// count, so that the regular tiles keep their XCD assignment (block index modulo the XCD
// count).  Where a row is short (the Chebyshev and update kernels) they come first and
// finish within the first round of blocks instead of trailing behind the tiles.
__host__ __device__ __forceinline__ int irr_blocks(int nrows, int rows_per_block)
{
    int nb = (nrows + rows_per_block - 1) / rows_per_block;
    return (nb + NXCD - 1) / NXCD * NXCD;
}


// ---------------------------------------------------------------------------------------
// B apply: v = B x (Eqs. A27 / As_qs at regular rows, A27_mod + C at irregular rows)
// ---------------------------------------------------------------------------------------
// Regular rows use sum factorisation of the tensor form
//   A = R_x (x) L_y (x) L_z + L_x (x) R_y (x) L_z + L_x (x) L_y (x) R_z
// with L = (a, 1, c) and R = (ar, br, cr) taken at the row's own index per direction
// (k_apply4 below, on vectorised rows).
//
// MODE_PLAIN  y = B x
// MODE_V      v = B x;  partials (w, v), (v, v);  finalize: alpha = rho / (r0, v)
// MODE_T      t = B x;  partials (t, w), (t, t);  finalize: omega = (t, s) / (t, t)
// MODE_RES    y = b - B x; partials (y, y), (y/d, y/d); finalize stores the norms
// `aux` is the second operand of the row's output: w[e] for MODE_V / MODE_T, b[e] for
// MODE_RES (unused for MODE_PLAIN).
template <typename T, int MODE>
using AuxT = typename std::conditional<MODE == MODE_RES, double, T>::type;

template <typename T, typename TO, int MODE>
__device__ __forceinline__ void emit(size_t e, T v, double bd, AuxT<T, MODE> aux, TO *__restrict__ y,
                                     double (&acc)[2])
{
    if (MODE == MODE_RES) {
        double r = (double)aux - (double)v;
        y[e] = (TO)r;
        double rd = r / bd;
        acc[0] += r * r;
        acc[1] += rd * rd;
    } else {
        y[e] = (TO)v;
        if (MODE == MODE_V || MODE == MODE_T) {
            acc[0] += (double)aux * (double)v;
            acc[1] += (double)v * (double)v;
        }
    }
}

template <typename T, int MODE>
__device__ __forceinline__ AuxT<T, MODE> load_aux(size_t e, const T *__restrict__ w, const double *__restrict__ bvec)
{
    if (MODE == MODE_RES) return bvec[e];
    if (MODE == MODE_V || MODE == MODE_T) return w[e];
    return AuxT<T, MODE>(0);
}

// One block: fixed-order totals of a reducing kernel's partials and the scalar updates of
// Alg. 1 that depend on them.
//   FIN_V       alpha = rho / (r0, v)        (breakdown when (r0, v) vanishes)
//   FIN_T       omega = (t, s) / (t, t)
//   FIN_UPDATE  rho_new = (r0, r); convergence on ||D^-1 r||; beta = (alpha/omega)(rho_new/rho)
//   FIN_RES     true residual norms ||r||^2, ||D^-1 r||^2
//   FIN_RESTART rho = r0n2 = (r, r); alpha = beta = 0, omega = 1
template <int KIND>
__global__ void __launch_bounds__(NT) k_finalize(const double *partials, int nblocks, DevState *st)
{
    constexpr int NV = (KIND == FIN_RESTART) ? 1 : 2;
    if ((KIND == FIN_V || KIND == FIN_T || KIND == FIN_UPDATE) && st->done) return;
    double tot[NV];
    total_partials<NV>(tot, partials, nblocks);
    if (threadIdx.x + threadIdx.y * blockDim.x != 0) return;
    if (KIND == FIN_V) {
        double sig = tot[0];
        if (!(sig == sig) || !(tot[NV - 1] == tot[NV - 1])) st->done = 3;
        else if (sig == 0.0 || fabs(sig) <= 1e-30 * sqrt(st->r0n2 * tot[NV - 1])) st->done = 2;
        else st->alpha = st->rho / sig;
    } else if (KIND == FIN_T) {
        double tt = tot[NV - 1];
        if (!(tt == tt) || !(tot[0] == tot[0])) st->done = 3;
        else st->omega = tt > 0.0 ? tot[0] / tt : 0.0;
    } else if (KIND == FIN_UPDATE) {
        double rho_new = tot[0];
        st->iters += 1;
        st->rn2s = tot[NV - 1];
        if (!(rho_new == rho_new) || !(tot[NV - 1] == tot[NV - 1])) st->done = 3;
        else if (tot[NV - 1] <= st->stop2) st->done = 1;
        else if (st->omega == 0.0 || st->rho == 0.0) st->done = 2;
        else {
            st->beta = (st->alpha / st->omega) * (rho_new / st->rho);
            st->rho = rho_new;
        }
    } else if (KIND == FIN_RES) {
        st->res2 = tot[0];
        st->res2s = tot[NV - 1];
    } else {
        st->rho = tot[0];
        st->r0n2 = tot[0];
        st->alpha = 0.0;
        st->beta = 0.0;
        st->omega = 1.0;
        st->rn2s = st->res2s;
        st->done = (tot[0] == tot[0]) ? ((st->res2s <= st->stop2) ? 1 : 0) : 3;
    }
}

// ---------------------------------------------------------------------------------------
// Chebyshev-Jacobi steps on K phi = rho (Sec. 3.3, Eqs. A7 / A7_mod)
// ---------------------------------------------------------------------------------------
// x_{m+1} = x_m + c1 (x_m - x_{m-1}) + c2 (rho - K x_m) / diag(K)
// (Chebyshev acceleration of Jacobi for -K, Saad Alg. 12.1), x_{m-1} = 0 when PREV0.
// Vectorised rows: a wavefront owns a 256-node segment of an x-row, four consecutive nodes
// per lane, loaded and stored as one 4-vector (rows start at any 4-byte boundary; the
// hardware splits unaligned vector accesses).  x neighbours come from the adjacent lanes;
// the two segment ends read theirs from memory.  A lane whose four nodes run past the row
// end (ragged rows) loads and stores its valid nodes one by one.
// ---------------------------------------------------------------------------------------
template <typename T>
struct Vec4Of;
template <>
struct Vec4Of<float> {
    typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct Vec4Of<double> {
    typedef double type __attribute__((ext_vector_type(4), aligned(8)));
};

// A wave-uniform value moved to a scalar register (it is the same in every lane).
__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The lane's nodes of a segment: i0 (first node), nv (valid nodes, <= 0 when none).
struct Seg {
    int i0, nv;
    bool full;
};

__device__ __forceinline__ Seg seg_of(int nx, int segment, int lane)
{
    Seg q;
    q.i0 = 1 + segment * (4 * TX) + 4 * lane;
    q.nv = min(4, nx - 1 - q.i0);
    q.full = q.nv == 4;
    return q;
}

// One 4-vector load for every lane, nodes past the row end zeroed by selects: a branch
// between a vector and a per-node path would make the compiler wait for all loads in
// flight at the join.  The last elements of a vector are followed by VEC_PAD zeros, so the
// four elements always lie inside the allocation.
template <typename T>
__device__ __forceinline__ typename Vec4Of<T>::type load4(const T *__restrict__ a, size_t e, const Seg &q)
{
    using V = typename Vec4Of<T>::type;
    V v = *reinterpret_cast<const V *>(a + e);
    if (q.nv < 4) {
        v.x = q.nv > 0 ? v.x : T(0);
        v.y = q.nv > 1 ? v.y : T(0);
        v.z = q.nv > 2 ? v.z : T(0);
        v.w = T(0);
    }
    return v;
}

// the four row-type bits of nodes i0 .. i0 + 3 (skip words are read in pairs; the array
// carries two words of padding)
__device__ __forceinline__ uint32_t skip4(const uint32_t *__restrict__ w, int i0)
{
    const uint64_t pair = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    return (uint32_t)(pair >> (i0 & 31)) & 0xFu;
}

// Single Chebyshev step on vectorised rows (same arithmetic as the per-node form):
//   x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 (rho - K x_k) / diag K
// Each wavefront owns RPW consecutive rows of a 256-node segment and marches in z.  At
// plane k it loads the rows' x_k at plane k + 1 (their upper z neighbours, and the centre
// of the next plane), the two outer y-neighbour rows, rho and x_{k-1}; the rows' x_k at
// planes k - 1 and k are carried in registers.  Latency is hidden by occupancy: issuing the
// loads of two or four planes before computing them (fewer waits per plane, more registers)
// measured no faster at 256^3, so the register budget goes to wavefronts and rows per
// wavefront.  Wave-uniform y and z coefficients live in scalar registers.  Irregular rows
// use their Shortley-Weller row in the leading blocks (one thread per row).  With RES the
// same rows give the residual rho - K x_k instead (multigrid), with no x_{k-1}.
// With MR (a coarse multigrid level whose rows fit in fewer than 64 lanes) each group of
// 2^g.lg lanes owns one whole row, so a wavefront carries 64 / 2^g.lg rows and no lane idles;
// the rows' y coefficients are then per lane.
template <typename T, bool PREV0, bool RES, bool REV, bool MR = false, int R = RPW>
__device__ __forceinline__ void cheb4_rows(const Geom &g, const Coef<T> &cf, const Irr<T> &ir,
                                           const uint32_t *__restrict__ skip, const T *__restrict__ xc,
                                           const T *xm1, const T *__restrict__ rho, T *xn, T c1, T c2,
                                           const DevState *st)
{
    using V = typename Vec4Of<T>::type;
    static_assert(!MR || R == 1, "multi-row wavefronts take one row per lane group");
    static_assert(R == RPW || R == RPW2, "the tilings hold these row counts");
    if (st && st->done) return;
    const int wv = threadIdx.y;
    const int lw = MR ? 1 << g.lg : TX;                          // lanes per row
    const int lane = MR ? (int)threadIdx.x & (lw - 1) : (int)threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t plane = (size_t)nx * ny;
    const int nib = irr_blocks(ir.n, NT);
    const int b = (int)blockIdx.x - nib;
    if (b < 0) {
        const int row = (int)blockIdx.x * NT + (int)threadIdx.x + wv * TX;
        if (row >= ir.n) return;
        const int e = ir.node[row];
        const T *k7 = ir.k7 + 7 * row;
        T z0 = xc[e];
        T kx = k7[0] * z0 + k7[1] * xc[e - 1] + k7[2] * xc[e + 1] + k7[3] * xc[e - nx] + k7[4] * xc[e + nx] +
               k7[5] * xc[e - plane] + k7[6] * xc[e + plane];
        T prev = PREV0 ? T(0) : xm1[e];
        xn[e] = RES ? rho[e] - kx : z0 + c1 * (z0 - prev) + c2 * (rho[e] - kx) / k7[0];
        return;
    }
    const Tiling &tl = (R == RPW) ? g.tr : tr2_of<T>(g);
    int bs, by, bz;
    if (!tile_of_block(tl, b, bs, by, bz)) return;
    const int jw = 1 + (by * TY + wv) * (MR ? TX / lw : R);    // the wavefront's first row
    if (jw > ny - 2) return;                                  // whole wavefront
    // rows j0 .. j0 + R - 1 (MR: one row per lane group, clamped to the wall row)
    const int j0 = MR ? min(jw + (int)threadIdx.x / lw, ny - 1) : jw;
    Seg q;
    if (MR) {
        q.i0 = 1 + bs * (4 * lw) + 4 * lane;
        q.nv = min(4, nx - 1 - q.i0);
        q.full = q.nv == 4;
    } else {
        q = seg_of(nx, bs, lane);
    }
    const int k0 = 1 + bz * tl.TZ;
    const int k1 = min(k0 + tl.TZ, nz - 1);
    const int ic = q.nv > 0 ? q.i0 : 1;                        // lanes without nodes read valid memory
    T kax[4], kbx[4], kcx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const T *cx = cf.c[0] + 8 * (u < q.nv ? q.i0 + u : 1);
        kax[u] = cx[5];
        kbx[u] = cx[6];
        kcx[u] = cx[7];
    }
    // rows past ny - 2 read the wall row ny - 1 (zero in every iterate: the right y
    // neighbour of the last interior row) and are not stored
    bool rok[R];
    size_t er[R], wr[R];
    T kay[R], kby[R], kcy[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        rok[r] = j <= ny - 2;
        const int jc = rok[r] ? j : ny - 1;
        er[r] = (size_t)ic + (size_t)nx * jc;
        wr[r] = (size_t)jc * g.W + (ic >> 5);
        kay[r] = MR ? cf.c[1][8 * jc + 5] : uniform(cf.c[1][8 * jc + 5]);
        kby[r] = MR ? cf.c[1][8 * jc + 6] : uniform(cf.c[1][8 * jc + 6]);
        kcy[r] = MR ? cf.c[1][8 * jc + 7] : uniform(cf.c[1][8 * jc + 7]);
    }
    const size_t elo = (size_t)ic + (size_t)nx * (j0 - 1);                  // row j0 - 1 (>= 0)
    const size_t ehi = (size_t)ic + (size_t)nx * min(j0 + R, ny - 1);       // row j0 + R (<= ny - 1)
    // the segment's outer neighbours: node i0 - 1 for lane 0, node i0 + nv for the last lane
    // (both walls, hence zero in every iterate, when one segment spans the row)
    const bool one_seg = nx - 2 <= 4 * lw;
    const bool need_l = lane == 0, need_r = lane == lw - 1 || q.i0 + 4 >= nx - 1;
    const int ir_off = q.nv > 0 ? q.nv : 0;
    const size_t wplane = (size_t)ny * g.W;

    // The march runs up in z, or down when rev is set: consecutive sweeps alternate, so that
    // each starts on the planes the previous one touched last (still in the caches).  `cb`
    // is the plane behind the march, `ca` the one ahead.
    constexpr int dir = REV ? -1 : 1;
    const int ks = REV ? k1 - 1 : k0;
    V cb[R], c0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        cb[r] = load4(xc, er[r] + (size_t)(ks - dir) * plane, q);
        c0[r] = load4(xc, er[r] + (size_t)ks * plane, q);
    }
    for (int t = 0; t < k1 - k0; ++t) {
        const int k = ks + dir * t;
        const size_t kp = (size_t)k * plane, kn = (size_t)(k + dir) * plane;
        V ca[R], rv4[R], pv4[R];
        uint32_t sk[R];
        T lft[R], rgt[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ca[r] = load4(xc, er[r] + kn, q);
            rv4[r] = load4(rho, er[r] + kp, q);
            if (!PREV0) pv4[r] = load4(xm1, er[r] + kp, q);
            sk[r] = skip4(skip + (size_t)k * wplane + wr[r], ic);
            lft[r] = (!one_seg && need_l) ? xc[er[r] + kp - 1] : T(0);
            rgt[r] = (!one_seg && need_r) ? xc[er[r] + kp + ir_off] : T(0);
        }
        const V ylo = load4(xc, elo + kp, q), yhi = load4(xc, ehi + kp, q);
        const T *cz = cf.c[2] + 8 * k;
        const T za = uniform(cz[5]), zb = uniform(cz[6]), zcc = uniform(cz[7]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const V &s4 = (r == 0) ? ylo : c0[r - 1];
            const V &n4 = (r == R - 1) ? yhi : c0[r + 1];
            const T cv[4] = {c0[r].x, c0[r].y, c0[r].z, c0[r].w};
            T left = MR ? __shfl_up(cv[3], 1, lw) : __shfl_up(cv[3], 1, TX);
            T right = MR ? __shfl_down(cv[0], 1, lw) : __shfl_down(cv[0], 1, TX);
            if (need_l) left = lft[r];
            if (need_r) right = rgt[r];
            const T sv[4] = {s4.x, s4.y, s4.z, s4.w};
            const T nvv[4] = {n4.x, n4.y, n4.z, n4.w};
            const V &lo4 = REV ? ca[r] : cb[r], &hi4 = REV ? cb[r] : ca[r];   // planes k - 1, k + 1
            const T mv[4] = {lo4.x, lo4.y, lo4.z, lo4.w};
            const T uv[4] = {hi4.x, hi4.y, hi4.z, hi4.w};
            const T rvv[4] = {rv4[r].x, rv4[r].y, rv4[r].z, rv4[r].w};
            T pv[4] = {T(0), T(0), T(0), T(0)};
            if (!PREV0) { pv[0] = pv4[r].x; pv[1] = pv4[r].y; pv[2] = pv4[r].z; pv[3] = pv4[r].w; }
            T out[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const T w = (u == 0) ? left : cv[u - 1];
                const T ea = (u + 1 < q.nv) ? cv[u + 1] : right;
                const T kd = kbx[u] + kby[r] + zb;
                const T kx = kd * cv[u] + kax[u] * w + kcx[u] * ea + kay[r] * sv[u] + kcy[r] * nvv[u] + za * mv[u] +
                             zcc * uv[u];
                out[u] = RES ? rvv[u] - kx : cv[u] + c1 * (cv[u] - pv[u]) + c2 * (rvv[u] - kx) / kd;
            }
            if (rok[r]) {
                const size_t e = er[r] + kp;
                if (q.full && sk[r] == 0u) {
                    V o = {out[0], out[1], out[2], out[3]};
                    *reinterpret_cast<V *>(xn + e) = o;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (u < q.nv && !((sk[r] >> u) & 1u)) xn[e + u] = out[u];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cb[r] = c0[r];
            c0[r] = ca[r];
        }
    }
}

template <typename T, bool PREV0, int R = RPW>
__global__ void __launch_bounds__(NT) k_cheb4(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                              const T *__restrict__ xc, const T *xm1,
                                              const T *__restrict__ rho, T *xn, T c1, T c2,
                                              const DevState *st, int rev)
{
    if (rev) cheb4_rows<T, PREV0, false, true, false, R>(g, cf, ir, skip, xc, xm1, rho, xn, c1, c2, st);
    else cheb4_rows<T, PREV0, false, false, false, R>(g, cf, ir, skip, xc, xm1, rho, xn, c1, c2, st);
}

// r = rho - K x at the unknown nodes (the residual of a multigrid level; same rows)
template <typename T, int R = RPW>
__global__ void __launch_bounds__(NT) k_resid4(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                               const T *__restrict__ x, const T *__restrict__ rho, T *r,
                                               const DevState *st, int rev)
{
    if (rev) cheb4_rows<T, true, true, true, false, R>(g, cf, ir, skip, x, nullptr, rho, r, T(0), T(0), st);
    else cheb4_rows<T, true, true, false, false, R>(g, cf, ir, skip, x, nullptr, rho, r, T(0), T(0), st);
}

// the same two kernels for coarse levels with several rows per wavefront (g.lg < 6)
template <typename T, bool PREV0>
__global__ void __launch_bounds__(NT) k_cheb4m(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                               const T *__restrict__ xc, const T *xm1,
                                               const T *__restrict__ rho, T *xn, T c1, T c2,
                                               const DevState *st, int rev)
{
    if (rev) cheb4_rows<T, PREV0, false, true, true>(g, cf, ir, skip, xc, xm1, rho, xn, c1, c2, st);
    else cheb4_rows<T, PREV0, false, false, true>(g, cf, ir, skip, xc, xm1, rho, xn, c1, c2, st);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_resid4m(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                                const T *__restrict__ x, const T *__restrict__ rho, T *r,
                                                const DevState *st, int rev)
{
    if (rev) cheb4_rows<T, true, true, true, true>(g, cf, ir, skip, x, nullptr, rho, r, T(0), T(0), st);
    else cheb4_rows<T, true, true, false, true>(g, cf, ir, skip, x, nullptr, rho, r, T(0), T(0), st);
}

// ---------------------------------------------------------------------------------------
// B apply on vectorised rows (modes above): a wavefront owns one
// row of a 256-node segment, four nodes per lane, and marches in z.  At plane kk it loads x
// of rows j - 1, j, j + 1 (the centre row's next plane from HBM, the outer rows mostly from
// L2), filters them along x (neighbours from the adjacent lanes) and then along y, keeping
// the y-filtered pairs (L_y L_x x, L_y R_x x + R_y L_x x) of planes kk - 2 .. kk; the z
// filter then gives row j at plane kk - 1.  No LDS and no barriers: latency is hidden by
// occupancy, as in the Chebyshev sweep (an LDS-staged 64 x 8 tile version with one barrier
// per plane measured no faster).  Irregular rows gather their stored full row of B in the
// blocks after the tiles, IRR_LANES lanes per row.
// ---------------------------------------------------------------------------------------
template <typename T, typename TO, int MODE>
__global__ void __launch_bounds__(NT) k_apply4(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                               const T *__restrict__ x, TO *__restrict__ y, const T *__restrict__ w,
                                               const double *__restrict__ bvec, DevState *st, double *partials)
{
    using V = typename Vec4Of<T>::type;
    constexpr int NV = (MODE == MODE_PLAIN) ? 0 : 2;
    if (MODE != MODE_PLAIN && MODE != MODE_RES && st->done) return;
    double acc[2] = {0.0, 0.0};
    const int lane = threadIdx.x, wv = threadIdx.y, tid = lane + wv * TX;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t plane = (size_t)nx * ny;
    // the irregular rows come after the tiles here: a full row of B is a gather of about 50
    // entries, and leading blocks of such rows held the tiles back (measured 65 against 52 us
    // per FP32 apply at 256^3 with 8 spheres)
    const int b = (int)blockIdx.x < g.ta.nblk ? (int)blockIdx.x : -1;
    const int irr_block = (int)blockIdx.x - g.ta.nblk;
    if (b >= 0) {
        const Tiling &tl = g.ta;
        int bs, by, bz;
        if (tile_of_block(tl, b, bs, by, bz) && 1 + by * TY + wv <= ny - 2) {
            const int jr = 1 + by * TY + wv;
            const Seg q = seg_of(nx, bs, lane);
            const int k0 = 1 + bz * tl.TZ;
            const int k1 = min(k0 + tl.TZ, nz - 1);               // output planes [k0, k1)
            const int ic = q.nv > 0 ? q.i0 : 1;
            T ax[4], cxx[4], arx[4], brx[4], crx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const T *cx = cf.c[0] + 8 * (u < q.nv ? q.i0 + u : 1);
                ax[u] = cx[0]; cxx[u] = cx[1]; arx[u] = cx[2]; brx[u] = cx[3]; crx[u] = cx[4];
            }
            const T *cy = cf.c[1] + 8 * jr;
            const T ay = uniform(cy[0]), cyy = uniform(cy[1]), ary = uniform(cy[2]), bry = uniform(cy[3]),
                    cry = uniform(cy[4]);
            const size_t e0 = (size_t)ic + (size_t)nx * jr;         // row j at plane 0
            const size_t wr = (size_t)jr * g.W + (ic >> 5);
            const size_t wplane = (size_t)ny * g.W;
            const bool one_seg = nx - 2 <= 4 * TX;
            const bool need_l = lane == 0, need_r = lane == TX - 1 || q.i0 + 4 >= nx - 1;
            const int ir_off = q.nv > 0 ? q.nv : 0;
            // x-filtered pair of one row at one plane: uL = L_x x, uR = R_x x
            auto xfilter = [&](const V &v4, T lft, T rgt, T (&uL)[4], T (&uR)[4]) __attribute__((always_inline)) {
                const T cv[4] = {v4.x, v4.y, v4.z, v4.w};
                T left = __shfl_up(cv[3], 1, TX), right = __shfl_down(cv[0], 1, TX);
                if (need_l) left = lft;
                if (need_r) right = rgt;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const T wm = (u == 0) ? left : cv[u - 1];
                    const T ep = (u + 1 < q.nv) ? cv[u + 1] : right;
                    uL[u] = ax[u] * wm + cv[u] + cxx[u] * ep;
                    uR[u] = arx[u] * wm + brx[u] * cv[u] + crx[u] * ep;
                }
            };
            T LL0[4], LR0[4], LL1[4], LR1[4];                       // planes kk - 2, kk - 1
#pragma unroll
            for (int u = 0; u < 4; ++u) LL0[u] = LR0[u] = LL1[u] = LR1[u] = T(0);
            for (int kk = k0 - 1; kk <= k1; ++kk) {
                const size_t kp = (size_t)kk * plane;
                const V xs = load4(x, e0 + kp - nx, q), xc = load4(x, e0 + kp, q), xn = load4(x, e0 + kp + nx, q);
                T ls = T(0), rs = T(0), lc = T(0), rc = T(0), ln = T(0), rn = T(0);
                if (!one_seg) {
                    if (need_l) { ls = x[e0 + kp - nx - 1]; lc = x[e0 + kp - 1]; ln = x[e0 + kp + nx - 1]; }
                    if (need_r) { rs = x[e0 + kp - nx + ir_off]; rc = x[e0 + kp + ir_off]; rn = x[e0 + kp + nx + ir_off]; }
                }
                // output plane k = kk - 1: row type bits and the second operand
                const int k = kk - 1;
                const bool out = k >= k0;
                const int kc = out ? k : k0;
                uint32_t sk = 0u;
                AuxT<T, MODE> aux[4];
                if (out) {
                    sk = skip4(skip + (size_t)kc * wplane + wr, ic);
                    if (MODE == MODE_RES) {
                        // b carries zero padding past its last node (one 4-vector load)
                        const typename Vec4Of<double>::type b4 = load4(bvec, e0 + (size_t)kc * plane, q);
                        aux[0] = b4.x; aux[1] = b4.y; aux[2] = b4.z; aux[3] = b4.w;
                    } else if (MODE == MODE_V || MODE == MODE_T) {
                        const V a4 = load4(w, e0 + (size_t)kc * plane, q);
                        aux[0] = a4.x; aux[1] = a4.y; aux[2] = a4.z; aux[3] = a4.w;
                    }
                }
                T sL[4], sR[4], cL[4], cR[4], nL[4], nR[4];
                xfilter(xs, ls, rs, sL, sR);
                xfilter(xc, lc, rc, cL, cR);
                xfilter(xn, ln, rn, nL, nR);
                T LL2[4], LR2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    LL2[u] = ay * sL[u] + cL[u] + cyy * nL[u];
                    LR2[u] = (ay * sR[u] + cR[u] + cyy * nR[u]) + (ary * sL[u] + bry * cL[u] + cry * nL[u]);
                }
                if (out) {
                    const T *cz = cf.c[2] + 8 * k;
                    const T az = uniform(cz[0]), ccz = uniform(cz[1]), arz = uniform(cz[2]), brz = uniform(cz[3]),
                            crz = uniform(cz[4]);
                    const size_t e = e0 + (size_t)k * plane;
                    TO o[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const T v = az * LR0[u] + LR1[u] + ccz * LR2[u] + arz * LL0[u] + brz * LL1[u] + crz * LL2[u];
                        const bool on = u < q.nv && !((sk >> u) & 1u);
                        if (MODE == MODE_RES) {
                            const double r = (double)aux[u] - (double)v, rd = r / (double)(brx[u] + bry + brz);
                            o[u] = (TO)r;
                            if (on) { acc[0] += r * r; acc[1] += rd * rd; }
                        } else {
                            o[u] = (TO)v;
                            if ((MODE == MODE_V || MODE == MODE_T) && on) {
                                acc[0] += (double)aux[u] * (double)v;
                                acc[1] += (double)v * (double)v;
                            }
                        }
                    }
                    // one 4-vector store where all four nodes are regular rows, else node by node
                    if (q.full && sk == 0u) {
                        typename Vec4Of<TO>::type ov = {o[0], o[1], o[2], o[3]};
                        *reinterpret_cast<typename Vec4Of<TO>::type *>(y + e) = ov;
                    } else {
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (u < q.nv && !((sk >> u) & 1u)) y[e + u] = o[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    LL0[u] = LL1[u]; LR0[u] = LR1[u];
                    LL1[u] = LL2[u]; LR1[u] = LR2[u];
                }
            }
        }
    } else {
        // irregular rows: IRR_LANES lanes per row gather the full row of B, four entries per
        // lane at a time (their column and value loads, then their x loads, are issued
        // together: three dependent memory round trips for a row of up to 64 entries)
        const int rows_per_block = NT / IRR_LANES;
        const int row = irr_block * rows_per_block + tid / IRR_LANES;
        const int il = tid % IRR_LANES;
        double sacc = 0.0;
        if (row < ir.n) {
            const int p0 = ir.ptr[row], p1 = ir.ptr[row + 1];
            for (int e = p0 + il; e < p1; e += 4 * IRR_LANES) {
                int c[4];
                T v[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int ee = e + t * IRR_LANES;
                    const int ec = ee < p1 ? ee : p0;       // entries past the row end read entry p0
                    c[t] = ir.col[ec];
                    const T vv = ir.val[ec];
                    v[t] = ee < p1 ? vv : T(0);
                }
                T xv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) xv[t] = x[c[t]];
#pragma unroll
                for (int t = 0; t < 4; ++t) sacc += (double)v[t] * (double)xv[t];
            }
        }
        for (int o = IRR_LANES / 2; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, IRR_LANES);
        if (row < ir.n && il == 0) {
            const size_t e = (size_t)ir.node[row];
            emit<T, TO, MODE>(e, (T)sacc, (double)ir.bdiag[row], load_aux<T, MODE>(e, w, bvec), y, acc);
        }
    }
    if constexpr (NV > 0) write_partials<2>(acc, partials);
}

// ---------------------------------------------------------------------------------------
// Vector updates of Alg. 1 on vectorised rows:
//   k_first4 FIRST_P  p = r + beta (p - omega v)   (search direction; p = r after a (re)start:
//                                                  beta = 0)
//            FIRST_S  s = r - alpha v              (intermediate residual)
//            then x_1 = c2 * (p or s) / diag(K), the first Chebyshev step from x_0 = 0
//   k_update4         u += alpha p^ + omega s^, r = s - omega t, partials of (r0, r) and of
//                     ||D^-1 r||^2 (D = diag B); the finalize kernel forms beta and tests
//                     convergence
// A wavefront owns one row of a 256-node segment, four nodes per lane, and walks its
// z-chunk.  The diagonals of K and B are formed from the 1D tables with the x coefficients
// held per lane and the y and z coefficients wave-uniform, so no node index is ever
// decoded.  Walls are not touched (zero in every vector); irregular rows (their own
// diagonals) run in the leading blocks, one thread per row.
// ---------------------------------------------------------------------------------------
template <typename T, int KIND>
__global__ void __launch_bounds__(NT) k_first4(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                               const T *__restrict__ r, T *__restrict__ ps, const T *__restrict__ v,
                                               T *__restrict__ x1, T c2, const DevState *st)
{
    using V = typename Vec4Of<T>::type;
    if (st->done) return;
    const T alpha = (T)st->alpha, beta = (T)st->beta, omega = (T)st->omega;
    const int lane = threadIdx.x, wv = threadIdx.y;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t plane = (size_t)nx * ny;
    const int nib = irr_blocks(ir.n, NT);
    const int b = (int)blockIdx.x - nib;
    if (b < 0) {
        const int row = (int)blockIdx.x * NT + (int)threadIdx.x + wv * TX;
        if (row >= ir.n) return;
        const int e = ir.node[row];
        const T val = (KIND == FIRST_P) ? r[e] + beta * (ps[e] - omega * v[e]) : r[e] - alpha * v[e];
        ps[e] = val;
        x1[e] = c2 * val / ir.k7[7 * row];
        return;
    }
    const Tiling &tl = g.ta;
    int bs, by, bz;
    if (!tile_of_block(tl, b, bs, by, bz)) return;
    const int jr = 1 + by * TY + wv;
    if (jr > ny - 2) return;
    const Seg q = seg_of(nx, bs, lane);
    const int ic = q.nv > 0 ? q.i0 : 1;
    const int k0 = 1 + bz * tl.TZ, k1 = min(k0 + tl.TZ, nz - 1);
    T kbx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) kbx[u] = cf.c[0][8 * (u < q.nv ? q.i0 + u : 1) + 6];
    const T kby = uniform(cf.c[1][8 * jr + 6]);
    const size_t e0 = (size_t)ic + (size_t)nx * jr, wr = (size_t)jr * g.W + (ic >> 5), wplane = (size_t)ny * g.W;
    for (int k = k0; k < k1; ++k) {
        const size_t e = e0 + (size_t)k * plane;
        const V r4 = load4(r, e, q), v4 = load4(v, e, q);
        V p4 = {T(0), T(0), T(0), T(0)};
        if (KIND == FIRST_P) p4 = load4(ps, e, q);
        const uint32_t sk = skip4(skip + (size_t)k * wplane + wr, ic);
        const T kz = uniform(cf.c[2][8 * k + 6]);
        const T rv[4] = {r4.x, r4.y, r4.z, r4.w}, vv[4] = {v4.x, v4.y, v4.z, v4.w}, pv[4] = {p4.x, p4.y, p4.z, p4.w};
        T out[4], xo[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            out[u] = (KIND == FIRST_P) ? rv[u] + beta * (pv[u] - omega * vv[u]) : rv[u] - alpha * vv[u];
            xo[u] = c2 * out[u] / (kbx[u] + kby + kz);
        }
        if (q.full && sk == 0u) {
            V o = {out[0], out[1], out[2], out[3]}, xq = {xo[0], xo[1], xo[2], xo[3]};
            *reinterpret_cast<V *>(ps + e) = o;
            *reinterpret_cast<V *>(x1 + e) = xq;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u < q.nv && !((sk >> u) & 1u)) {
                    ps[e + u] = out[u];
                    x1[e + u] = xo[u];
                }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(NT) k_update4(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                                T *__restrict__ xs, const T *__restrict__ ph, const T *__restrict__ sh,
                                                const T *__restrict__ s, const T *__restrict__ t,
                                                const T *__restrict__ r0, T *__restrict__ r, DevState *st,
                                                double *partials)
{
    using V = typename Vec4Of<T>::type;
    if (st->done) return;
    const T alphaT = (T)st->alpha, omegaT = (T)st->omega;
    double acc[2] = {0.0, 0.0};
    const int lane = threadIdx.x, wv = threadIdx.y;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t plane = (size_t)nx * ny;
    const int nib = irr_blocks(ir.n, NT);
    const int b = (int)blockIdx.x - nib;
    if (b < 0) {
        // irregular rows: x and r are updated by the tiles like every node; here only the
        // Jacobi-weighted norm with the row's own diagonal
        const int row = (int)blockIdx.x * NT + (int)threadIdx.x + wv * TX;
        if (row < ir.n) {
            const int e = ir.node[row];
            const T rv = s[e] - omegaT * t[e];
            const double rd = (double)rv / (double)ir.bdiag[row];
            acc[1] += rd * rd;
        }
    } else {
        const Tiling &tl = g.ta;
        int bs, by, bz;
        const bool tile = tile_of_block(tl, b, bs, by, bz);
        const int jr = tile ? 1 + by * TY + wv : ny;
        if (jr <= ny - 2) {
            const Seg q = seg_of(nx, bs, lane);
            const int ic = q.nv > 0 ? q.i0 : 1;
            const int k0 = 1 + bz * tl.TZ, k1 = min(k0 + tl.TZ, nz - 1);
            T brx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) brx[u] = cf.c[0][8 * (u < q.nv ? q.i0 + u : 1) + 3];
            const T bry = uniform(cf.c[1][8 * jr + 3]);
            const size_t e0 = (size_t)ic + (size_t)nx * jr, wr = (size_t)jr * g.W + (ic >> 5),
                         wplane = (size_t)ny * g.W;
            for (int k = k0; k < k1; ++k) {
                const size_t e = e0 + (size_t)k * plane;
                const V x4 = load4(xs, e, q), p4 = load4(ph, e, q), h4 = load4(sh, e, q), s4 = load4(s, e, q),
                        t4 = load4(t, e, q), z4 = load4(r0, e, q);
                const uint32_t sk = skip4(skip + (size_t)k * wplane + wr, ic);
                const T brz = uniform(cf.c[2][8 * k + 3]);
                const T xv[4] = {x4.x, x4.y, x4.z, x4.w}, pv[4] = {p4.x, p4.y, p4.z, p4.w},
                        hv[4] = {h4.x, h4.y, h4.z, h4.w}, sv[4] = {s4.x, s4.y, s4.z, s4.w},
                        tv[4] = {t4.x, t4.y, t4.z, t4.w}, zv[4] = {z4.x, z4.y, z4.z, z4.w};
                T xo[4], ro[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xo[u] = xv[u] + (alphaT * pv[u] + omegaT * hv[u]);
                    ro[u] = sv[u] - omegaT * tv[u];
                    if (u < q.nv) {
                        acc[0] += (double)zv[u] * (double)ro[u];
                        if (!((sk >> u) & 1u)) {
                            const double rd = (double)ro[u] / ((double)brx[u] + (double)bry + (double)brz);
                            acc[1] += rd * rd;
                        }
                    }
                }
                if (q.full) {
                    V xq = {xo[0], xo[1], xo[2], xo[3]}, rq = {ro[0], ro[1], ro[2], ro[3]};
                    *reinterpret_cast<V *>(xs + e) = xq;
                    *reinterpret_cast<V *>(r + e) = rq;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (u < q.nv) {
                            xs[e + u] = xo[u];
                            r[e + u] = ro[u];
                        }
                }
            }
        }
    }
    write_partials<2>(acc, partials);
}

// ---------------------------------------------------------------------------------------
// flat pointwise kernels: threads stride over all nodes in groups of 16 bytes; wall and
// solid entries are 0 in every vector and stay 0
// ---------------------------------------------------------------------------------------
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float4 type;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    typedef double2 type;
    static constexpr int n = 2;
};

template <typename T>
__device__ __forceinline__ void load16(const T *p, T (&v)[Vec16<T>::n])
{
    typename Vec16<T>::type q = *reinterpret_cast<const typename Vec16<T>::type *>(p);
    const T *a = reinterpret_cast<const T *>(&q);
#pragma unroll
    for (int u = 0; u < Vec16<T>::n; ++u) v[u] = a[u];
}

template <typename T>
__device__ __forceinline__ void store16(T *p, const T (&v)[Vec16<T>::n])
{
    typename Vec16<T>::type q;
    T *a = reinterpret_cast<T *>(&q);
#pragma unroll
    for (int u = 0; u < Vec16<T>::n; ++u) a[u] = v[u];
    *reinterpret_cast<typename Vec16<T>::type *>(p) = q;
}

// (re)start: r0 = r, p = v = 0, rho = (r, r); the recursive norm starts from the true one
template <typename T>
__global__ void __launch_bounds__(NT) k_restart(Geom g, const T *__restrict__ r, T *__restrict__ r0, T *__restrict__ p,
                                                T *__restrict__ v, DevState *st, double *partials,
                                                int nblocks)
{
    constexpr int VN = Vec16<T>::n;
    double acc[1] = {0.0};
    const int tid = threadIdx.x + threadIdx.y * TX;
    const size_t nn = (size_t)g.nx * g.ny * g.nz;
    const size_t ngroups = nn / VN;
    for (size_t q = (size_t)blockIdx.x * NT + tid; q < ngroups; q += (size_t)gridDim.x * NT) {
        const size_t base = q * VN;
        T rv[VN], z[VN];
        load16(r + base, rv);
#pragma unroll
        for (int u = 0; u < VN; ++u) {
            z[u] = T(0);
            acc[0] += (double)rv[u] * (double)rv[u];
        }
        store16(r0 + base, rv);
        store16(p + base, z);
        store16(v + base, z);
    }
    write_partials<1>(acc, partials);
}

// u64 += d32 (refinement step) on unknown rows; d is exactly 0 elsewhere
__global__ void k_add_correction(size_t n, double *__restrict__ u, const float *__restrict__ d)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e < n; e += (size_t)gridDim.x * blockDim.x) u[e] += (double)d[e];
}

template <typename T>
__global__ void k_fill(size_t n, T *__restrict__ a, T val)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e < n; e += (size_t)gridDim.x * blockDim.x) a[e] = val;
}

// 0 in every vector of the list at the nodes that are not unknowns (types other than 1 and 2)
// and in the padding past the last node; the unknowns' entries are left as they are
template <typename T>
__global__ void k_zero_off_unknowns(size_t nn, size_t pad, const int8_t *__restrict__ type, VecList<T> v)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e < nn + pad; e += (size_t)gridDim.x * blockDim.x) {
        if (e < nn) {
            const int8_t t = type[e];
            if (t == 1 || t == 2) continue;
        }
        for (int q = 0; q < v.n; ++q) v.p[q][e] = T(0);
    }
}

// dst = src at unknown nodes (types 1, 2), 0 elsewhere; converts precision
template <typename TI, typename TO>
__global__ void k_masked_copy(size_t n, const int8_t *__restrict__ type, const TI *__restrict__ src, TO *__restrict__ dst)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e < n; e += (size_t)gridDim.x * blockDim.x) {
        int8_t t = type[e];
        dst[e] = (t == 1 || t == 2) ? (TO)src[e] : TO(0);
    }
}

// output u: unknowns from x, wall nodes g, solid nodes 0
__global__ void k_output(size_t n, const int8_t *__restrict__ type, const double *__restrict__ x,
                         const double *__restrict__ gv, double *__restrict__ u)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e < n; e += (size_t)gridDim.x * blockDim.x) {
        int8_t t = type[e];
        u[e] = (t == 1 || t == 2) ? x[e] : (t == 0 ? gv[e] : 0.0);
    }
}

// 1 if any unknown entry is not finite
__global__ void k_check_finite(size_t n, const int8_t *__restrict__ type, const double *__restrict__ x, int *flag)
{
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e < n; e += (size_t)gridDim.x * blockDim.x) {
        int8_t t = type[e];
        if ((t == 1 || t == 2) && !isfinite(x[e])) atomicOr(flag, 1);
    }
}

// Per-block partial sums (a, b) and (b, b) over the unknown nodes, in a fixed order; the
// host adds the DOT_BLOCKS partials in block order.
__global__ void __launch_bounds__(256) k_dot2_unknowns(size_t n, const int8_t *__restrict__ type,
                                                       const double *__restrict__ a, const double *__restrict__ b,
                                                       double *__restrict__ partials)
{
    __shared__ double sh[2][256 / 64];
    double acc[2] = {0.0, 0.0};
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const int8_t t = type[e];
        if (t == 1 || t == 2) {
            acc[0] += a[e] * b[e];
            acc[1] += b[e] * b[e];
        }
    }
    for (int q = 0; q < 2; ++q) acc[q] = wave_sum(acc[q]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { sh[0][wv] = acc[0]; sh[1][wv] = acc[1]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < 256 / 64; ++w) { s0 += sh[0][w]; s1 += sh[1][w]; }
        partials[2 * blockIdx.x] = s0;
        partials[2 * blockIdx.x + 1] = s1;
    }
}

__global__ void k_scale(size_t n, double *__restrict__ x, double alpha)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        x[e] *= alpha;
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
static inline dim3 tile_block() { return dim3(TX, TY, 1); }

template <int KIND>
static void finalize(const Launch &L, int nb, DevState *st)
{
    k_finalize<KIND><<<1, tile_block(), 0, L.stream>>>(L.partials, nb, st);
}

template <typename T, typename TO>
void launch_apply(int mode, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *x, TO *y, const T *w,
                  const double *bvec, DevState *st)
{
    int nb = L.g.ta.nblk + irr_blocks(ir.n, NT / IRR_LANES);
    dim3 grid(nb), blk = tile_block();
#define CPS_APPLY_LAUNCH(M) \
    k_apply4<T, TO, M><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials)
    switch (mode) {
    case MODE_PLAIN:
        CPS_APPLY_LAUNCH(MODE_PLAIN);
        break;
    case MODE_V:
        CPS_APPLY_LAUNCH(MODE_V);
        finalize<FIN_V>(L, nb, st);
        break;
    case MODE_T:
        CPS_APPLY_LAUNCH(MODE_T);
        finalize<FIN_T>(L, nb, st);
        break;
    case MODE_RES:
        CPS_APPLY_LAUNCH(MODE_RES);
        finalize<FIN_RES>(L, nb, st);
        break;
    }
#undef CPS_APPLY_LAUNCH
}

template <typename T>
void launch_cheb(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *xc, const T *xm1, const T *rho, T *xn,
                 double c1, double c2, const DevState *st, int rev, hipEvent_t ev0, hipEvent_t ev1)
{
    dim3 grid(L.g.tr.nblk + irr_blocks(ir.n, NT)), blk = tile_block();
    const bool mr = L.g.lg < 6;
    if (xm1 == nullptr) {
        // the sweep without an x_{k-1} moves less per plane step: RPW2 rows per wavefront
        dim3 grid2(tr2_of<T>(L.g).nblk + irr_blocks(ir.n, NT));
        if (mr) k_cheb4m<T, true><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st, rev);
        else if (ev0)
            hipExtLaunchKernelGGL((k_cheb4<T, true, RPW2>), grid2, blk, 0, L.stream, ev0, ev1, 0, L.g, cf, ir, L.skip, xc,
                                  xm1, rho, xn, (T)c1, (T)c2, st, rev);
        else k_cheb4<T, true, RPW2><<<grid2, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st,
                                                               rev);
    } else {
        if (mr) k_cheb4m<T, false><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st, rev);
        else if (ev0)
            hipExtLaunchKernelGGL((k_cheb4<T, false>), grid, blk, 0, L.stream, ev0, ev1, 0, L.g, cf, ir, L.skip, xc, xm1,
                                  rho, xn, (T)c1, (T)c2, st, rev);
        else k_cheb4<T, false><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st, rev);
    }
}

template <typename T>
void launch_resid(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *x, const T *rho, T *r,
                  const DevState *st, int rev)
{
    dim3 grid(L.g.tr.nblk + irr_blocks(ir.n, NT)), blk = tile_block();
    dim3 grid2(tr2_of<T>(L.g).nblk + irr_blocks(ir.n, NT));
    if (L.g.lg < 6) k_resid4m<T><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, rho, r, st, rev);
    else k_resid4<T, RPW2><<<grid2, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, rho, r, st, rev);
}

template <typename T>
void launch_resid_irregular(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *x, const T *rho, T *r,
                            const DevState *st)
{
    // a grid of irregular-row blocks only: no tile work
    const int nib = irr_blocks(ir.n, NT);
    if (nib > 0) k_resid4<T, RPW2><<<dim3(nib), tile_block(), 0, L.stream>>>(L.g, cf, ir, L.skip, x, rho, r, st, 0);
}

template <typename T>
void launch_first(int kind, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *r, T *ps, const T *v, T *x1,
                  double c2, const DevState *st)
{
    dim3 grid(L.g.ta.nblk + irr_blocks(ir.n, NT)), blk = tile_block();
    if (kind == FIRST_P)
        k_first4<T, FIRST_P><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, r, ps, v, x1, (T)c2, st);
    else
        k_first4<T, FIRST_S><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, r, ps, v, x1, (T)c2, st);
}

template <typename T, typename TX_>
void launch_update(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, TX_ *xs, const T *ph, const T *sh, const T *s,
                   const T *t, const T *r0, T *r, DevState *st)
{
    static_assert(sizeof(T) == sizeof(TX_), "solution and Krylov vectors share a precision");
    int nb = L.g.ta.nblk + irr_blocks(ir.n, NT);
    k_update4<T><<<dim3(nb), tile_block(), 0, L.stream>>>(L.g, cf, ir, L.skip, (T *)xs, ph, sh, s, t, r0, r, st,
                                                          L.partials);
    finalize<FIN_UPDATE>(L, nb, st);
}

template <typename T>
void launch_restart(const Launch &L, const Irr<T> &ir, const T *r, T *r0, T *p, T *v, DevState *st)
{
    int nb = L.g.nflat;
    k_restart<T><<<dim3(nb), tile_block(), 0, L.stream>>>(L.g, r, r0, p, v, st, L.partials, nb);
    finalize<FIN_RESTART>(L, nb, st);
}

static inline dim3 flat_grid(size_t n) { return dim3((unsigned)std::min<size_t>((n + 255) / 256, 65536)); }

void launch_add_correction(hipStream_t s, size_t n, double *u, const float *d)
{
    k_add_correction<<<flat_grid(n), 256, 0, s>>>(n, u, d);
}

template <typename T>
void launch_zero_off_unknowns(hipStream_t s, size_t nn, size_t pad, const int8_t *type, const VecList<T> &v)
{
    if (v.n > 0) k_zero_off_unknowns<T><<<flat_grid(nn + pad), 256, 0, s>>>(nn, pad, type, v);
}

template <typename T>
void launch_fill(hipStream_t s, size_t n, T *a, T val)
{
    k_fill<T><<<flat_grid(n), 256, 0, s>>>(n, a, val);
}

template <typename TI, typename TO>
void launch_masked_copy(hipStream_t s, size_t n, const int8_t *type, const TI *src, TO *dst)
{
    k_masked_copy<TI, TO><<<flat_grid(n), 256, 0, s>>>(n, type, src, dst);
}

void launch_output(hipStream_t s, size_t n, const int8_t *type, const double *x, const double *gv, double *u)
{
    k_output<<<flat_grid(n), 256, 0, s>>>(n, type, x, gv, u);
}

void launch_check_finite(hipStream_t s, size_t n, const int8_t *type, const double *x, int *flag)
{
    k_check_finite<<<flat_grid(n), 256, 0, s>>>(n, type, x, flag);
}

void launch_dot2_unknowns(hipStream_t s, size_t n, const int8_t *type, const double *a, const double *b,
                          double *partials)
{
    k_dot2_unknowns<<<DOT_BLOCKS, 256, 0, s>>>(n, type, a, b, partials);
}

void launch_scale(hipStream_t s, size_t n, double *x, double alpha)
{
    k_scale<<<flat_grid(n), 256, 0, s>>>(n, x, alpha);
}

// explicit instantiations
template void launch_apply<double, double>(int, const Launch &, const Coef<double> &, const Irr<double> &,
                                           const double *, double *, const double *, const double *, DevState *);
template void launch_apply<double, float>(int, const Launch &, const Coef<double> &, const Irr<double> &,
                                          const double *, float *, const double *, const double *, DevState *);
template void launch_apply<float, float>(int, const Launch &, const Coef<float> &, const Irr<float> &, const float *,
                                         float *, const float *, const double *, DevState *);
template void launch_cheb<double>(const Launch &, const Coef<double> &, const Irr<double> &, const double *,
                                  const double *, const double *, double *, double, double, const DevState *, int,
                                  hipEvent_t, hipEvent_t);
template void launch_cheb<float>(const Launch &, const Coef<float> &, const Irr<float> &, const float *, const float *,
                                 const float *, float *, double, double, const DevState *, int, hipEvent_t, hipEvent_t);
template void launch_resid_irregular<double>(const Launch &, const Coef<double> &, const Irr<double> &,
                                             const double *, const double *, double *, const DevState *);
template void launch_resid_irregular<float>(const Launch &, const Coef<float> &, const Irr<float> &, const float *,
                                            const float *, float *, const DevState *);
template void launch_resid<double>(const Launch &, const Coef<double> &, const Irr<double> &, const double *,
                                   const double *, double *, const DevState *, int);
template void launch_resid<float>(const Launch &, const Coef<float> &, const Irr<float> &, const float *, const float *,
                                  float *, const DevState *, int);
template void launch_first<double>(int, const Launch &, const Coef<double> &, const Irr<double> &, const double *,
                                   double *, const double *, double *, double, const DevState *);
template void launch_first<float>(int, const Launch &, const Coef<float> &, const Irr<float> &, const float *, float *,
                                  const float *, float *, double, const DevState *);
template void launch_update<double, double>(const Launch &, const Coef<double> &, const Irr<double> &, double *,
                                            const double *, const double *, const double *, const double *,
                                            const double *, double *, DevState *);
template void launch_update<float, float>(const Launch &, const Coef<float> &, const Irr<float> &, float *, const float *,
                                          const float *, const float *, const float *, const float *, float *,
                                          DevState *);
template void launch_restart<double>(const Launch &, const Irr<double> &, const double *, double *, double *, double *,
                                     DevState *);
template void launch_restart<float>(const Launch &, const Irr<float> &, const float *, float *, float *, float *,
                                    DevState *);
template void launch_zero_off_unknowns<double>(hipStream_t, size_t, size_t, const int8_t *, const VecList<double> &);
template void launch_zero_off_unknowns<float>(hipStream_t, size_t, size_t, const int8_t *, const VecList<float> &);
template void launch_fill<double>(hipStream_t, size_t, double *, double);
template void launch_fill<float>(hipStream_t, size_t, float *, float);
template void launch_fill<unsigned>(hipStream_t, size_t, unsigned *, unsigned);
template void launch_masked_copy<double, double>(hipStream_t, size_t, const int8_t *, const double *, double *);
template void launch_masked_copy<double, float>(hipStream_t, size_t, const int8_t *, const double *, float *);
template void launch_masked_copy<float, double>(hipStream_t, size_t, const int8_t *, const float *, double *);

}  // namespace cps
