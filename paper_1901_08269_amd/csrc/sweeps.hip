// sweeps.hip -- the hot path of the solve: the matrix-free compact operator B (regular rows
// in tiles, irregular rows from their table in the same launch), the Chebyshev-Jacobi
// sweeps of the preconditioner K, and the BiCGSTAB vector updates with their dot products
// reduced in the same launch (Alg. 1 with the split of Eq. Bdec).
//
// Launch shape: the stencil kernels use 64 x 4 (Chebyshev) or 64 x 8 (B apply) column
// tiles of the interior that march over z-chunks (XCD-aware tile order); the pointwise
// kernels stride over all nodes with 16-byte vectors; blocks ahead of those process the
// irregular rows.  Kernels that reduce write one partial per block; a one-block finalize
// kernel that follows sums them in a fixed order (deterministic) and updates the
// device-resident BiCGSTAB scalars, so the host never waits inside an iteration.
#include "cps_device.h"
#include "cps_kernels.h"

namespace cps {

// Blocks that process irregular rows come first in every launch that has them, in a count
// rounded up to a multiple of the XCD count: they are short, so they finish within the
// first round of blocks instead of trailing behind the regular tiles, and the regular
// tiles keep their XCD assignment (block index modulo the XCD count).
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
// with L = (a, 1, c) and R = (ar, br, cr) taken at the row's own index per direction.
// A block owns a 64 x 8 column tile (two rows per thread) and marches in z: each plane of x
// (with a one-node halo) is staged in a double-buffered LDS tile while the next two planes
// are already being fetched into registers; every thread filters its 3 x 3 neighbourhood along
// x, then y, from LDS and keeps the two y-filtered planes it still needs in registers.
// One barrier per plane.
//
// MODE_PLAIN  y = B x
// MODE_V      v = B x;  partials (w, v), (v, v);  finalize: alpha = rho / (r0, v)
// MODE_T      t = B x;  partials (t, w), (t, t);  finalize: omega = (t, s) / (t, t)
// MODE_RES    y = b - B x; partials (y, y), (y/d, y/d); finalize stores the norms
// `aux` is the second operand of the row's output: w[e] for MODE_V / MODE_T, b[e] for
// MODE_RES (unused for MODE_PLAIN).  The regular tiles load it one pipeline stage ahead.
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

template <typename T, typename TO, int MODE>
__global__ void __launch_bounds__(NT) k_apply(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                              const T *__restrict__ x, TO *__restrict__ y, const T *__restrict__ w,
                                              const double *__restrict__ bvec, DevState *st, double *partials,
                                              unsigned *ticket, int nblocks)
{
    constexpr int NV = (MODE == MODE_PLAIN) ? 0 : 2;
    constexpr int AY = 2 * TY;                       // tile rows (two per thread)
    constexpr int LW = TX + 2, LH = AY + 2;          // staged plane with a one-node halo
    constexpr int NLD = (LW * LH + NT - 1) / NT;     // staging loads per thread and plane
    if (MODE != MODE_PLAIN && MODE != MODE_RES && st->done) return;
    __shared__ T su[2][LH][LW];
    double acc[2] = {0.0, 0.0};
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ty * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t plane = (size_t)nx * ny;
    const int nib = irr_blocks(ir.n, NT / IRR_LANES);
    const int b = (int)blockIdx.x - nib;
    const Tiling &tl = g.t8;
    if (b >= 0) {
        int bx, by, bz;
        if (tile_of_block(tl, b, bx, by, bz)) {
            const int x0 = 1 + bx * TX, y0 = 1 + by * AY;
            const int i = x0 + tx, ja = y0 + ty, jb = ja + TY;
            const int k0 = 1 + bz * tl.TZ;
            const int k1 = min(k0 + tl.TZ, g.nz - 1);      // output planes [k0, k1)
            const bool iok = i <= nx - 2, aok = iok && ja <= ny - 2, bok = iok && jb <= ny - 2;
            // x-filtered values are computed per thread, so coefficients only need to be
            // valid where they are used; out-of-range columns/rows read index 1
            const T *cx = cf.c[0] + 8 * (iok ? i : 1);
            const T *ca = cf.c[1] + 8 * (ja <= ny - 2 ? ja : 1);
            const T *cb = cf.c[1] + 8 * (jb <= ny - 2 ? jb : 1);
            const T ax = cx[0], ccx = cx[1], arx = cx[2], brx = cx[3], crx = cx[4];
            const T aya = ca[0], cya = ca[1], arya = ca[2], brya = ca[3], crya = ca[4];
            const T ayb = cb[0], cyb = cb[1], aryb = cb[2], bryb = cb[3], cryb = cb[4];
            // staging slots of this thread
            int soff[NLD], srow[NLD], scol[NLD];
            bool sok[NLD], sin[NLD];
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                int idx = tid + q * NT;
                sin[q] = idx < LW * LH;
                int r = sin[q] ? idx / LW : 0, c = sin[q] ? idx - r * LW : 0;
                srow[q] = r;
                scol[q] = c;
                int gi = x0 - 1 + c, gj = y0 - 1 + r;
                sok[q] = sin[q] && gi < nx && gj < ny;
                soff[q] = sok[q] ? gi + nx * gj : 0;
            }
            // Two register sets serve alternate planes.  While plane kk sits in LDS, planes
            // kk+1 and kk+2 of x are in flight, together with the skip words and the second
            // operand (aux) of the output rows two steps ahead.  Every load of a step is
            // issued after the waits of that step, so the in-order completion counter never
            // forces a wait on a plane that is still being prefetched.  The loop is unrolled
            // by two so that each set and each LDS buffer has a fixed role and no in-flight
            // register is ever copied.
            using AT = AuxT<T, MODE>;
            struct Set { T r[NLD]; AT wa, wb; uint32_t sa, sb; T z[5]; };
            Set A, B;
            // lanes outside the grid address row 1, column 1 and are masked off by aok / bok
            const int ic = iok ? i : 1;
            const size_t ea0 = (size_t)ic + (size_t)nx * (aok ? ja : 1), eb0 = (size_t)ic + (size_t)nx * (bok ? jb : 1);
            const uint32_t *ska = skip + (size_t)(aok ? ja : 1) * g.W + (ic >> 5);
            const uint32_t *skb = skip + (size_t)(bok ? jb : 1) * g.W + (ic >> 5);
            const size_t skw = (size_t)g.ny * g.W;
            // x of plane kk (clamped to k1; planes past k1 are loaded but unused)
            auto stage_fetch = [&](Set &S, int kk) __attribute__((always_inline)) {
                const size_t kp = (size_t)min(kk, k1) * plane;
#pragma unroll
                for (int q = 0; q < NLD; ++q) S.r[q] = sok[q] ? x[(size_t)soff[q] + kp] : T(0);
            };
            // row-type bits, aux and z coefficients of output plane k (clamped to k1 - 1)
            auto aux_fetch = [&](Set &S, int k) __attribute__((always_inline)) {
                k = min(k, k1 - 1);
                const size_t kp = (size_t)k * plane;
                S.sa = aok ? ska[(size_t)k * skw] : ~0u;
                S.sb = bok ? skb[(size_t)k * skw] : ~0u;
                if (MODE != MODE_PLAIN) {
                    S.wa = load_aux<T, MODE>(ea0 + kp, w, bvec);
                    S.wb = load_aux<T, MODE>(eb0 + kp, w, bvec);
                }
                const T *cz = cf.c[2] + 8 * k;
#pragma unroll
                for (int q = 0; q < 5; ++q) S.z[q] = cz[q];
            };
            stage_fetch(A, k0 - 1);
            stage_fetch(B, k0);
            A.wa = A.wb = B.wa = B.wb = AT(0);
            A.sa = A.sb = B.sa = B.sb = ~0u;
#pragma unroll
            for (int q = 0; q < 5; ++q) A.z[q] = B.z[q] = T(0);
            T LLa0 = 0, LRa0 = 0, LLa1 = 0, LRa1 = 0, LLb0 = 0, LRb0 = 0, LLb1 = 0, LRb1 = 0;
            auto plane_step = [&](Set &S, T (&lds)[LH][LW], int kk) __attribute__((always_inline)) {
#pragma unroll
                for (int q = 0; q < NLD; ++q)
                    if (sin[q]) lds[srow[q]][scol[q]] = S.r[q];
                stage_fetch(S, kk + 2);
                __syncthreads();
                // x filters of the three rows around row a (LDS rows ty..ty+2) and row b
                T ul[6], ur[6];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    T um = lds[ty + r][tx], u0 = lds[ty + r][tx + 1], up = lds[ty + r][tx + 2];
                    ul[r] = ax * um + u0 + ccx * up;
                    ur[r] = arx * um + brx * u0 + crx * up;
                    T vm = lds[ty + TY + r][tx], v0 = lds[ty + TY + r][tx + 1], vp = lds[ty + TY + r][tx + 2];
                    ul[3 + r] = ax * vm + v0 + ccx * vp;
                    ur[3 + r] = arx * vm + brx * v0 + crx * vp;
                }
                T LLa2 = aya * ul[0] + ul[1] + cya * ul[2];
                T LRa2 = (aya * ur[0] + ur[1] + cya * ur[2]) + (arya * ul[0] + brya * ul[1] + crya * ul[2]);
                T LLb2 = ayb * ul[3] + ul[4] + cyb * ul[5];
                T LRb2 = (ayb * ur[3] + ur[4] + cyb * ur[5]) + (aryb * ul[3] + bryb * ul[4] + cryb * ul[5]);
                if (kk >= k0 + 1) {
                    const int k = kk - 1;
                    const size_t kp = (size_t)k * plane;
                    const T az = S.z[0], ccz = S.z[1], arz = S.z[2], brz = S.z[3], crz = S.z[4];
                    if (!((S.sa >> (i & 31)) & 1u)) {
                        T v = az * LRa0 + LRa1 + ccz * LRa2 + arz * LLa0 + brz * LLa1 + crz * LLa2;
                        emit<T, TO, MODE>(ea0 + kp, v, (double)(brx + brya + brz), S.wa, y, acc);
                    }
                    if (!((S.sb >> (i & 31)) & 1u)) {
                        T v = az * LRb0 + LRb1 + ccz * LRb2 + arz * LLb0 + brz * LLb1 + crz * LLb2;
                        emit<T, TO, MODE>(eb0 + kp, v, (double)(brx + bryb + brz), S.wb, y, acc);
                    }
                }
                aux_fetch(S, kk + 1);
                LLa0 = LLa1; LRa0 = LRa1; LLa1 = LLa2; LRa1 = LRa2;
                LLb0 = LLb1; LRb0 = LRb1; LLb1 = LLb2; LRb1 = LRb2;
            };
            for (int kk = k0 - 1; kk <= k1; kk += 2) {
                plane_step(A, su[0], kk);
                if (kk + 1 > k1) break;
                plane_step(B, su[1], kk + 1);
            }
        }
    } else {
        // irregular rows: IRR_LANES lanes per row gather the full row of B
        const int rows_per_block = NT / IRR_LANES;
        const int row = (int)blockIdx.x * rows_per_block + tid / IRR_LANES;
        const int lane = tid % IRR_LANES;
        double sacc = 0.0;
        if (row < ir.n) {
            for (int e = ir.ptr[row] + lane; e < ir.ptr[row + 1]; e += IRR_LANES)
                sacc += (double)ir.val[e] * (double)x[ir.col[e]];
        }
        for (int o = IRR_LANES / 2; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, IRR_LANES);
        if (row < ir.n && lane == 0) {
            const size_t e = (size_t)ir.node[row];
            emit<T, TO, MODE>(e, (T)sacc, (double)ir.bdiag[row], load_aux<T, MODE>(e, w, bvec), y, acc);
        }
    }
    if constexpr (NV > 0) write_partials<2>(acc, partials);
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
// Regular rows: K from the second-order 1D tables.  Each thread marches its column in z
// with the three z-neighbours in registers and every operand of the next plane already in
// flight while the current plane is computed; x and y neighbours come through L1.
// Irregular rows use their stored Shortley-Weller row (one thread per row, same launch).
template <typename T, bool PREV0>
__global__ void __launch_bounds__(NT) k_cheb(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                             const T *__restrict__ xc, const T *__restrict__ xm1,
                                             const T *__restrict__ rho, T *__restrict__ xn, T c1, T c2,
                                             const DevState *st)
{
    if (st && st->done) return;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ty * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t plane = (size_t)nx * ny;
    const int nib = irr_blocks(ir.n, NT);
    const int b = (int)blockIdx.x - nib;
    const Tiling &tl = g.t4;
    if (b >= 0) {
        int bx, by, bz;
        if (!tile_of_block(tl, b, bx, by, bz)) return;
        const int i = 1 + bx * TX + tx, j = 1 + by * TY + ty;
        if (i > nx - 2 || j > ny - 2) return;
        const int k0 = 1 + bz * tl.TZ;
        const int k1 = min(k0 + tl.TZ, g.nz - 1);
        const T *cx = cf.c[0] + 8 * i;
        const T *cy = cf.c[1] + 8 * j;
        const T kax = cx[5], kbx = cx[6], kcx = cx[7];
        const T kay = cy[5], kby = cy[6], kcy = cy[7];
        const size_t e0 = (size_t)i + (size_t)nx * j;
        // Software pipeline over three register sets, one per plane: plane k is computed
        // from sets (k-1, k, k+1) and the set of plane k-1, dead after that, then receives
        // plane k+2, so two planes of loads stay in flight.  Every operand of a plane (its
        // skip word and z coefficients included) travels in its set: a load issued just
        // before its use would make the in-order completion counter wait for the whole
        // prefetch.  Fetches are unconditional, with the plane clamped to k1 <= nz - 1
        // (planes past k1 are loaded but unused), and the loop is unrolled by three so that
        // each set keeps a fixed register home.
        struct Pl { T c, w, e, s, n, r, p, za, zb, zc; uint32_t sk; };
        const size_t skw = (size_t)g.ny * g.W;
        const uint32_t *skp = skip + (size_t)j * g.W + (i >> 5);
        auto fetch = [&](Pl &P, int k) __attribute__((always_inline)) {
            k = min(k, k1);
            const size_t e = e0 + (size_t)k * plane;
            const T *cz = cf.c[2] + 8 * k;
            P.sk = skp[(size_t)k * skw];
            P.c = xc[e];
            P.w = xc[e - 1];
            P.e = xc[e + 1];
            P.s = xc[e - nx];
            P.n = xc[e + nx];
            P.r = rho[e];
            P.p = PREV0 ? T(0) : xm1[e];
            P.za = cz[5];
            P.zb = cz[6];
            P.zc = cz[7];
        };
        auto step = [&](const Pl &M, const Pl &C, const Pl &U, Pl &F, int k) __attribute__((always_inline)) {
            T kd = kbx + kby + C.zb;
            T kx = kd * C.c + kax * C.w + kcx * C.e + kay * C.s + kcy * C.n + C.za * M.c + C.zc * U.c;
            T val = C.c + c1 * (C.c - C.p) + c2 * (C.r - kx) / kd;
            if (!((C.sk >> (i & 31)) & 1u)) xn[e0 + (size_t)k * plane] = val;
            fetch(F, k + 2);
        };
        Pl P0, P1, P2;
        fetch(P2, k0 - 1);
        fetch(P0, k0);
        fetch(P1, k0 + 1);
        for (int k = k0; k < k1; k += 3) {
            step(P2, P0, P1, P2, k);
            if (k + 1 >= k1) break;
            step(P0, P1, P2, P0, k + 1);
            if (k + 2 >= k1) break;
            step(P1, P2, P0, P1, k + 2);
        }
    } else {
        const int row = (int)blockIdx.x * NT + tid;
        if (row >= ir.n) return;
        const int e = ir.node[row];
        const T *k7 = ir.k7 + 7 * row;
        T z0 = xc[e];
        T kx = k7[0] * z0 + k7[1] * xc[e - 1] + k7[2] * xc[e + 1] + k7[3] * xc[e - nx] + k7[4] * xc[e + nx] +
               k7[5] * xc[e - plane] + k7[6] * xc[e + plane];
        T prev = PREV0 ? T(0) : xm1[e];
        xn[e] = z0 + c1 * (z0 - prev) + c2 * (rho[e] - kx) / k7[0];
    }
}

// ---------------------------------------------------------------------------------------
// flat, vectorised pointwise kernels: blocks [0, nflat) stride over all nodes in groups of
// 16 bytes per thread; wall and solid entries are 0 in every vector and stay 0
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

// node coordinates of `base` and its successors
struct NodeIt {
    int i, j, k;
    __device__ NodeIt(size_t base, int nx, int ny)
    {
        i = (int)(base % nx);
        size_t r = base / nx;
        j = (int)(r % ny);
        k = (int)(r / ny);
    }
    __device__ void next(int nx, int ny)
    {
        if (++i == nx) {
            i = 0;
            if (++j == ny) { j = 0; ++k; }
        }
    }
};

// FIRST_P:  p = r + beta (p - omega v)   (search direction of Alg. 1; p = r after a (re)start: beta = 0)
// FIRST_S:  s = r - alpha v              (intermediate residual of Alg. 1)
// then x1 = c2 * (p or s) / diag(K), the first Chebyshev step from x0 = 0.  Irregular rows
// (their K diagonal is the Shortley-Weller one) are done by the leading blocks.
template <typename T, int KIND>
__global__ void __launch_bounds__(NT) k_first(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                              const T *__restrict__ r, T *__restrict__ ps, const T *__restrict__ v,
                                              T *__restrict__ x1, T c2, const DevState *st)
{
    if (st->done) return;
    constexpr int VN = Vec16<T>::n;
    const T alpha = (T)st->alpha, beta = (T)st->beta, omega = (T)st->omega;
    const int tid = threadIdx.x + threadIdx.y * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t nn = (size_t)nx * ny * g.nz;
    const int nib = irr_blocks(ir.n, NT);
    const int b = (int)blockIdx.x - nib;
    if (b >= 0) {
        const size_t ngroups = nn / VN;
        for (size_t q = (size_t)b * NT + tid; q < ngroups; q += (size_t)g.nflat * NT) {
            const size_t base = q * VN;
            T rv[VN], pv[VN], vv[VN], out[VN], xo[VN];
            load16(r + base, rv);
            load16(v + base, vv);
            if (KIND == FIRST_P) load16(ps + base, pv);
            NodeIt it(base, nx, ny);
            bool any_skip = false;
#pragma unroll
            for (int u = 0; u < VN; ++u) {
                out[u] = (KIND == FIRST_P) ? rv[u] + beta * (pv[u] - omega * vv[u]) : rv[u] - alpha * vv[u];
                T kd = cf.c[0][8 * it.i + 6] + cf.c[1][8 * it.j + 6] + cf.c[2][8 * it.k + 6];
                xo[u] = c2 * out[u] / kd;
                any_skip |= skip_bit(skip, g, it.i, it.j, it.k);
                it.next(nx, ny);
            }
            if (!any_skip) {
                store16(ps + base, out);
                store16(x1 + base, xo);
            } else {
                NodeIt it2(base, nx, ny);
#pragma unroll
                for (int u = 0; u < VN; ++u) {
                    if (!skip_bit(skip, g, it2.i, it2.j, it2.k)) {
                        ps[base + u] = out[u];
                        x1[base + u] = xo[u];
                    }
                    it2.next(nx, ny);
                }
            }
        }
        // tail nodes (nn not a multiple of VN) are wall nodes: nothing to do
    } else {
        const int row = (int)blockIdx.x * NT + tid;
        if (row >= ir.n) return;
        const int e = ir.node[row];
        T val = (KIND == FIRST_P) ? r[e] + beta * (ps[e] - omega * v[e]) : r[e] - alpha * v[e];
        ps[e] = val;
        x1[e] = c2 * val / ir.k7[7 * row];
    }
}

// Solution and residual updates of Alg. 1: x += alpha p^ + omega s^, r = s - omega t, partials of (r0, r) and of
// ||D^-1 r||^2 (D = diag B; regular rows in the flat part, irregular rows by the leading
// blocks); the finalize kernel forms beta and tests convergence.
template <typename T>
__global__ void __launch_bounds__(NT) k_update(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                               T *__restrict__ xs, const T *__restrict__ ph, const T *__restrict__ sh,
                                               const T *__restrict__ s, const T *__restrict__ t,
                                               const T *__restrict__ r0, T *__restrict__ r, DevState *st,
                                               double *partials, unsigned *ticket, int nblocks)
{
    if (st->done) return;
    constexpr int VN = Vec16<T>::n;
    const double alpha = st->alpha, omega = st->omega;
    const T alphaT = (T)alpha, omegaT = (T)omega;
    double acc[2] = {0.0, 0.0};
    const int tid = threadIdx.x + threadIdx.y * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t nn = (size_t)nx * ny * g.nz;
    const int nib = irr_blocks(ir.n, NT);
    const int b = (int)blockIdx.x - nib;
    if (b >= 0) {
        const size_t ngroups = nn / VN;
        for (size_t q = (size_t)b * NT + tid; q < ngroups; q += (size_t)g.nflat * NT) {
            const size_t base = q * VN;
            T xv[VN], pv[VN], shv[VN], sv[VN], tv[VN], r0v[VN], rv[VN];
            load16(xs + base, xv);
            load16(ph + base, pv);
            load16(sh + base, shv);
            load16(s + base, sv);
            load16(t + base, tv);
            load16(r0 + base, r0v);
            NodeIt it(base, nx, ny);
#pragma unroll
            for (int u = 0; u < VN; ++u) {
                xv[u] = xv[u] + (alphaT * pv[u] + omegaT * shv[u]);
                rv[u] = sv[u] - omegaT * tv[u];
                acc[0] += (double)r0v[u] * (double)rv[u];
                if (!skip_bit(skip, g, it.i, it.j, it.k)) {
                    double d = (double)cf.c[0][8 * it.i + 3] + (double)cf.c[1][8 * it.j + 3] + (double)cf.c[2][8 * it.k + 3];
                    double rd = (double)rv[u] / d;
                    acc[1] += rd * rd;
                }
                it.next(nx, ny);
            }
            store16(xs + base, xv);
            store16(r + base, rv);
        }
    } else {
        const int row = (int)blockIdx.x * NT + tid;
        if (row < ir.n) {
            const int e = ir.node[row];
            T rv = s[e] - omegaT * t[e];
            double rd = (double)rv / (double)ir.bdiag[row];
            acc[1] += rd * rd;
        }
    }
    write_partials<2>(acc, partials);
}

// (re)start: r0 = r, p = v = 0, rho = (r, r); the recursive norm starts from the true one
template <typename T>
__global__ void __launch_bounds__(NT) k_restart(Geom g, const T *__restrict__ r, T *__restrict__ r0, T *__restrict__ p,
                                                T *__restrict__ v, DevState *st, double *partials, unsigned *ticket,
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
    int nb = L.g.t8.nblk + irr_blocks(ir.n, NT / IRR_LANES);
    dim3 grid(nb), blk = tile_block();
    switch (mode) {
    case MODE_PLAIN:
        k_apply<T, TO, MODE_PLAIN><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        break;
    case MODE_V:
        k_apply<T, TO, MODE_V><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        finalize<FIN_V>(L, nb, st);
        break;
    case MODE_T:
        k_apply<T, TO, MODE_T><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        finalize<FIN_T>(L, nb, st);
        break;
    case MODE_RES:
        k_apply<T, TO, MODE_RES><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        finalize<FIN_RES>(L, nb, st);
        break;
    }
}

template <typename T>
void launch_cheb(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *xc, const T *xm1, const T *rho, T *xn,
                 double c1, double c2, const DevState *st)
{
    dim3 grid(L.g.t4.nblk + irr_blocks(ir.n, NT)), blk = tile_block();
    if (xm1 == nullptr)
        k_cheb<T, true><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st);
    else
        k_cheb<T, false><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st);
}

template <typename T>
void launch_first(int kind, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *r, T *ps, const T *v, T *x1,
                  double c2, const DevState *st)
{
    dim3 grid(L.g.nflat + irr_blocks(ir.n, NT)), blk = tile_block();
    if (kind == FIRST_P)
        k_first<T, FIRST_P><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, r, ps, v, x1, (T)c2, st);
    else
        k_first<T, FIRST_S><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, r, ps, v, x1, (T)c2, st);
}

template <typename T, typename TX_>
void launch_update(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, TX_ *xs, const T *ph, const T *sh, const T *s,
                   const T *t, const T *r0, T *r, DevState *st)
{
    static_assert(sizeof(T) == sizeof(TX_), "solution and Krylov vectors share a precision");
    int nb = L.g.nflat + irr_blocks(ir.n, NT);
    k_update<T><<<dim3(nb), tile_block(), 0, L.stream>>>(L.g, cf, ir, L.skip, (T *)xs, ph, sh, s, t, r0, r, st,
                                                         L.partials, L.ticket, nb);
    finalize<FIN_UPDATE>(L, nb, st);
}

template <typename T>
void launch_restart(const Launch &L, const Irr<T> &ir, const T *r, T *r0, T *p, T *v, DevState *st)
{
    int nb = L.g.nflat;
    k_restart<T><<<dim3(nb), tile_block(), 0, L.stream>>>(L.g, r, r0, p, v, st, L.partials, L.ticket, nb);
    finalize<FIN_RESTART>(L, nb, st);
}

static inline dim3 flat_grid(size_t n) { return dim3((unsigned)std::min<size_t>((n + 255) / 256, 65536)); }

void launch_add_correction(hipStream_t s, size_t n, double *u, const float *d)
{
    k_add_correction<<<flat_grid(n), 256, 0, s>>>(n, u, d);
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

// explicit instantiations
template void launch_apply<double, double>(int, const Launch &, const Coef<double> &, const Irr<double> &,
                                           const double *, double *, const double *, const double *, DevState *);
template void launch_apply<double, float>(int, const Launch &, const Coef<double> &, const Irr<double> &,
                                          const double *, float *, const double *, const double *, DevState *);
template void launch_apply<float, float>(int, const Launch &, const Coef<float> &, const Irr<float> &, const float *,
                                         float *, const float *, const double *, DevState *);
template void launch_cheb<double>(const Launch &, const Coef<double> &, const Irr<double> &, const double *,
                                  const double *, const double *, double *, double, double, const DevState *);
template void launch_cheb<float>(const Launch &, const Coef<float> &, const Irr<float> &, const float *, const float *,
                                 const float *, float *, double, double, const DevState *);
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
template void launch_fill<double>(hipStream_t, size_t, double *, double);
template void launch_fill<float>(hipStream_t, size_t, float *, float);
template void launch_fill<unsigned>(hipStream_t, size_t, unsigned *, unsigned);
template void launch_masked_copy<double, double>(hipStream_t, size_t, const int8_t *, const double *, double *);
template void launch_masked_copy<double, float>(hipStream_t, size_t, const int8_t *, const double *, float *);
template void launch_masked_copy<float, double>(hipStream_t, size_t, const int8_t *, const float *, double *);

}  // namespace cps
