// sweeps.hip -- the hot path of the solve: the matrix-free compact operator B (regular rows
// in tiles, irregular rows from their table in the same launch), the Chebyshev-Jacobi
// sweeps of the preconditioner K, and the BiCGSTAB vector updates with their dot products
// reduced in the same launch (Alg. 1 with the split of Eq. Bdec).
//
// Launch shape of every kernel here: blocks [0, nblk_tiles) are (64 x 4) tiles of the
// interior that march over a z-chunk of TZ planes (XCD-aware tile order); blocks beyond
// that process the irregular rows.  Kernels that reduce write one partial per block; the
// last block to finish sums them in a fixed order (deterministic) and updates the
// device-resident BiCGSTAB scalars, so the host never waits inside an iteration.
#include "cps_device.h"
#include "cps_kernels.h"

namespace cps {

// ---------------------------------------------------------------------------------------
// B apply: v = B x (Eqs. A27 / As_qs at regular rows, A27_mod + C at irregular rows)
// ---------------------------------------------------------------------------------------
// Regular rows use sum factorisation of the tensor form
//   A = R_x (x) L_y (x) L_z + L_x (x) R_y (x) L_z + L_x (x) L_y (x) R_z
// with L = (a, 1, c) and R = (ar, br, cr) taken at the row's own index per direction:
// per z-plane the block stages x in LDS, filters along x (L_x u, R_x u), then along y,
// and keeps the three y-filtered planes it needs in registers while it marches in z.
//
// MODE_PLAIN  y = B x
// MODE_V      v = B x;  partials (w, v), (v, v);  last block: alpha = rho / (r0, v)
// MODE_T      t = B x;  partials (t, w), (t, t);  last block: omega = (t, s) / (t, t)
// MODE_RES    y = b - B x; partials (y, y), (y/d, y/d); last block stores the norms
template <typename T, typename TO, int MODE>
__global__ void __launch_bounds__(NT) k_apply(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                              const T *__restrict__ x, TO *__restrict__ y, const T *__restrict__ w,
                                              const double *__restrict__ bvec, DevState *st, double *partials,
                                              unsigned *ticket, int nblocks)
{
    constexpr int NV = (MODE == MODE_PLAIN) ? 0 : 2;
    if (MODE != MODE_PLAIN && MODE != MODE_RES && st->done) return;
    __shared__ T su[TY + 2][TX + 2];
    __shared__ T sL[TY + 2][TX];
    __shared__ T sR[TY + 2][TX];
    double acc[2] = {0.0, 0.0};
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ty * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t plane = (size_t)nx * ny;
    const int b = blockIdx.x;
    if (b < g.nblk_tiles) {
        int bx, by, bz;
        if (tile_of_block(g, b, bx, by, bz)) {
            const int x0 = 1 + bx * TX, y0 = 1 + by * TY;
            const int i = x0 + tx, j = y0 + ty;
            const int k0 = 1 + bz * g.TZ;
            const int k1 = min(k0 + g.TZ, g.nz - 1);      // output planes [k0, k1)
            const bool own = (i <= nx - 2) && (j <= ny - 2);
            // x-filtered rows are shared through LDS by every row of the tile, so the x
            // coefficients depend on i alone (and the y ones on j alone)
            const T *cx = cf.c[0] + 8 * (i <= nx - 2 ? i : 1);
            const T *cy = cf.c[1] + 8 * (j <= ny - 2 ? j : 1);
            const T ax = cx[0], ccx = cx[1], arx = cx[2], brx = cx[3], crx = cx[4];
            const T ay = cy[0], ccy = cy[1], ary = cy[2], bry = cy[3], cry = cy[4];
            T LL0 = 0, LR0 = 0, LL1 = 0, LR1 = 0;   // y-filtered planes k-1 and k
            for (int kk = k0 - 1; kk <= k1; ++kk) {
                const T *xp = x + (size_t)kk * plane;
                for (int q = tid; q < (TY + 2) * (TX + 2); q += NT) {
                    int r = q / (TX + 2), c = q - r * (TX + 2);
                    int gi = x0 - 1 + c, gj = y0 - 1 + r;
                    su[r][c] = (gi < nx && gj < ny) ? xp[gi + (size_t)nx * gj] : T(0);
                }
                __syncthreads();
                for (int r = ty; r < TY + 2; r += TY) {
                    T um = su[r][tx], u0 = su[r][tx + 1], up = su[r][tx + 2];
                    sL[r][tx] = ax * um + u0 + ccx * up;
                    sR[r][tx] = arx * um + brx * u0 + crx * up;
                }
                __syncthreads();
                T l_m = sL[ty][tx], l_0 = sL[ty + 1][tx], l_p = sL[ty + 2][tx];
                T r_m = sR[ty][tx], r_0 = sR[ty + 1][tx], r_p = sR[ty + 2][tx];
                T LL2 = ay * l_m + l_0 + ccy * l_p;                 // L_y L_x u
                T LR2 = (ay * r_m + r_0 + ccy * r_p)                // L_y R_x u
                        + (ary * l_m + bry * l_0 + cry * l_p);      // + R_y L_x u
                if (kk >= k0 + 1) {
                    const int k = kk - 1;
                    const T *cz = cf.c[2] + 8 * k;
                    const T az = cz[0], ccz = cz[1], arz = cz[2], brz = cz[3], crz = cz[4];
                    if (own && !skip_bit(skip, g, i, j, k)) {
                        T v = az * LR0 + LR1 + ccz * LR2 + arz * LL0 + brz * LL1 + crz * LL2;
                        size_t e = (size_t)i + (size_t)nx * j + (size_t)k * plane;
                        if (MODE == MODE_RES) {
                            double r = bvec[e] - (double)v;
                            y[e] = (TO)r;
                            double rd = r / (double)(brx + bry + brz);
                            acc[0] += r * r;
                            acc[1] += rd * rd;
                        } else {
                            y[e] = (TO)v;
                            if (MODE == MODE_V) {
                                acc[0] += (double)w[e] * (double)v;
                                acc[1] += (double)v * (double)v;
                            } else if (MODE == MODE_T) {
                                acc[0] += (double)v * (double)w[e];
                                acc[1] += (double)v * (double)v;
                            }
                        }
                    }
                }
                LL0 = LL1; LR0 = LR1;
                LL1 = LL2; LR1 = LR2;
            }
        }
    } else {
        // irregular rows: IRR_LANES lanes per row gather the full row of B
        const int rows_per_block = NT / IRR_LANES;
        const int row = (b - g.nblk_tiles) * rows_per_block + tid / IRR_LANES;
        const int lane = tid % IRR_LANES;
        double s = 0.0;
        if (row < ir.n) {
            for (int e = ir.ptr[row] + lane; e < ir.ptr[row + 1]; e += IRR_LANES)
                s += (double)ir.val[e] * (double)x[ir.col[e]];
        }
        for (int o = IRR_LANES / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, IRR_LANES);
        if (row < ir.n && lane == 0) {
            const int e = ir.node[row];
            if (MODE == MODE_RES) {
                double r = bvec[e] - s;
                y[e] = (TO)r;
                double rd = r / (double)ir.bdiag[row];
                acc[0] += r * r;
                acc[1] += rd * rd;
            } else {
                T v = (T)s;
                y[e] = (TO)v;
                if (MODE == MODE_V) {
                    acc[0] += (double)w[e] * (double)v;
                    acc[1] += (double)v * (double)v;
                } else if (MODE == MODE_T) {
                    acc[0] += (double)v * (double)w[e];
                    acc[1] += (double)v * (double)v;
                }
            }
        }
    }
    if constexpr (NV > 0) {
        if (publish_partials<2>(acc, partials, ticket, nblocks)) {
            double tot[2];
            total_partials<2>(tot, partials, ticket, nblocks);
            if (tid == 0) {
                if (MODE == MODE_V) {
                    // alpha = (r0, r_i) / (r0, v), Alg. 1; breakdown when (r0, v) vanishes
                    double sig = tot[0];
                    if (!(sig == sig) || !(tot[1] == tot[1])) st->done = 3;
                    else if (sig == 0.0 || fabs(sig) <= 1e-30 * sqrt(st->r0n2 * tot[1])) st->done = 2;
                    else st->alpha = st->rho / sig;
                } else if (MODE == MODE_T) {
                    // omega = (t, s) / (t, t)
                    double tt = tot[1];
                    if (!(tt == tt) || !(tot[0] == tot[0])) st->done = 3;
                    else st->omega = tt > 0.0 ? tot[0] / tt : 0.0;
                } else if (MODE == MODE_RES) {
                    st->res2 = tot[0];
                    st->res2s = tot[1];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Chebyshev-Jacobi steps on K phi = rho (Sec. 3.3, Eqs. A7 / A7_mod)
// ---------------------------------------------------------------------------------------
// x_{m+1} = x_m + c1 (x_m - x_{m-1}) + c2 (rho - K x_m) / diag(K)
// (Chebyshev acceleration of Jacobi for -K, Saad Alg. 12.1), x_{m-1} = 0 when PREV0.
// Regular rows: K from the second-order 1D tables; the z neighbours stay in registers
// while the column marches in z; x and y neighbours come from L1.  Irregular rows use
// their stored Shortley-Weller row (one thread per row, same launch).
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
    const int b = blockIdx.x;
    if (b < g.nblk_tiles) {
        int bx, by, bz;
        if (!tile_of_block(g, b, bx, by, bz)) return;
        const int i = 1 + bx * TX + tx, j = 1 + by * TY + ty;
        if (i > nx - 2 || j > ny - 2) return;
        const int k0 = 1 + bz * g.TZ;
        const int k1 = min(k0 + g.TZ, g.nz - 1);
        const T *cx = cf.c[0] + 8 * i;
        const T *cy = cf.c[1] + 8 * j;
        const T kax = cx[5], kbx = cx[6], kcx = cx[7];
        const T kay = cy[5], kby = cy[6], kcy = cy[7];
        size_t e = (size_t)i + (size_t)nx * j + (size_t)k0 * plane;
        T zm = xc[e - plane], z0 = xc[e];
        for (int k = k0; k < k1; ++k, e += plane) {
            T zp = xc[e + plane];
            if (!skip_bit(skip, g, i, j, k)) {
                const T *cz = cf.c[2] + 8 * k;
                T kd = kbx + kby + cz[6];
                T kx = kd * z0 + kax * xc[e - 1] + kcx * xc[e + 1] + kay * xc[e - nx] + kcy * xc[e + nx] +
                       cz[5] * zm + cz[7] * zp;
                T prev = PREV0 ? T(0) : xm1[e];
                xn[e] = z0 + c1 * (z0 - prev) + c2 * (rho[e] - kx) / kd;
            }
            zm = z0;
            z0 = zp;
        }
    } else {
        const int row = (b - g.nblk_tiles) * NT + tid;
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
// pointwise updates of Alg. 1 fused with the first Chebyshev step (x_1 = c2 rho / diag K)
// ---------------------------------------------------------------------------------------
// FIRST_P:  p = r + beta (p - omega v)   (line 14; p = r after a (re)start: beta = 0)
// FIRST_S:  s = r - alpha v              (line 7)
// then x1 = c2 * (p or s) / diag(K) into `x1`.
template <typename T, int KIND>
__global__ void __launch_bounds__(NT) k_first(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                              const T *__restrict__ r, T *__restrict__ ps, const T *__restrict__ v,
                                              T *__restrict__ x1, T c2, const DevState *st)
{
    if (st->done) return;
    const T alpha = (T)st->alpha, beta = (T)st->beta, omega = (T)st->omega;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ty * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t plane = (size_t)nx * ny;
    const int b = blockIdx.x;
    if (b < g.nblk_tiles) {
        int bx, by, bz;
        if (!tile_of_block(g, b, bx, by, bz)) return;
        const int i = 1 + bx * TX + tx, j = 1 + by * TY + ty;
        if (i > nx - 2 || j > ny - 2) return;
        const int k0 = 1 + bz * g.TZ;
        const int k1 = min(k0 + g.TZ, g.nz - 1);
        const T kbxy = cf.c[0][8 * i + 6] + cf.c[1][8 * j + 6];
        size_t e = (size_t)i + (size_t)nx * j + (size_t)k0 * plane;
        for (int k = k0; k < k1; ++k, e += plane) {
            if (skip_bit(skip, g, i, j, k)) continue;
            T val = (KIND == FIRST_P) ? r[e] + beta * (ps[e] - omega * v[e]) : r[e] - alpha * v[e];
            ps[e] = val;
            x1[e] = c2 * val / (kbxy + cf.c[2][8 * k + 6]);
        }
    } else {
        const int row = (b - g.nblk_tiles) * NT + tid;
        if (row >= ir.n) return;
        const int e = ir.node[row];
        T val = (KIND == FIRST_P) ? r[e] + beta * (ps[e] - omega * v[e]) : r[e] - alpha * v[e];
        ps[e] = val;
        x1[e] = c2 * val / ir.k7[7 * row];
    }
}

// ---------------------------------------------------------------------------------------
// lines 11-13 of Alg. 1: x += alpha p^ + omega s^, r = s - omega t, (r0, r), ||D^-1 r||^2
// ---------------------------------------------------------------------------------------
template <typename T, typename TX_>
__global__ void __launch_bounds__(NT) k_update(Geom g, Coef<T> cf, Irr<T> ir, const uint32_t *__restrict__ skip,
                                               TX_ *__restrict__ xs, const T *__restrict__ ph,
                                               const T *__restrict__ sh, const T *__restrict__ s,
                                               const T *__restrict__ t, const T *__restrict__ r0, T *__restrict__ r,
                                               DevState *st, double *partials, unsigned *ticket, int nblocks)
{
    if (st->done) return;
    const double alpha = st->alpha, omega = st->omega;
    const T alphaT = (T)alpha, omegaT = (T)omega;
    double acc[2] = {0.0, 0.0};
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ty * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t plane = (size_t)nx * ny;
    const int b = blockIdx.x;
    if (b < g.nblk_tiles) {
        int bx, by, bz;
        if (tile_of_block(g, b, bx, by, bz)) {
            const int i = 1 + bx * TX + tx, j = 1 + by * TY + ty;
            if (i <= nx - 2 && j <= ny - 2) {
                const int k0 = 1 + bz * g.TZ;
                const int k1 = min(k0 + g.TZ, g.nz - 1);
                const T bxy = cf.c[0][8 * i + 3] + cf.c[1][8 * j + 3];
                size_t e = (size_t)i + (size_t)nx * j + (size_t)k0 * plane;
                for (int k = k0; k < k1; ++k, e += plane) {
                    if (skip_bit(skip, g, i, j, k)) continue;
                    xs[e] = (TX_)((double)xs[e] + (double)(alphaT * ph[e] + omegaT * sh[e]));
                    T rv = s[e] - omegaT * t[e];
                    r[e] = rv;
                    double rd = (double)rv / (double)(bxy + cf.c[2][8 * k + 3]);
                    acc[0] += (double)r0[e] * (double)rv;
                    acc[1] += rd * rd;
                }
            }
        }
    } else {
        const int row = (b - g.nblk_tiles) * NT + tid;
        if (row < ir.n) {
            const int e = ir.node[row];
            xs[e] = (TX_)((double)xs[e] + (double)(alphaT * ph[e] + omegaT * sh[e]));
            T rv = s[e] - omegaT * t[e];
            r[e] = rv;
            double rd = (double)rv / (double)ir.bdiag[row];
            acc[0] += (double)r0[e] * (double)rv;
            acc[1] += rd * rd;
        }
    }
    if (publish_partials<2>(acc, partials, ticket, nblocks)) {
        double tot[2];
        total_partials<2>(tot, partials, ticket, nblocks);
        if (tid == 0) {
            double rho_new = tot[0];
            st->iters += 1;
            st->rn2s = tot[1];
            if (!(rho_new == rho_new) || !(tot[1] == tot[1])) {
                st->done = 3;
            } else if (tot[1] <= st->stop2) {
                st->done = 1;
            } else if (omega == 0.0 || st->rho == 0.0) {
                st->done = 2;
            } else {
                st->beta = (alpha / omega) * (rho_new / st->rho);   // line 13
                st->rho = rho_new;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// (re)start: r0 = r, p = v = 0, rho = (r, r), recursive norm from the true residual norms
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NT) k_restart(Geom g, Irr<T> ir, const uint32_t *__restrict__ skip,
                                                const T *__restrict__ r, T *__restrict__ r0, T *__restrict__ p,
                                                T *__restrict__ v, DevState *st, double *partials, unsigned *ticket,
                                                int nblocks)
{
    double acc[1] = {0.0};
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ty * TX;
    const int nx = g.nx, ny = g.ny;
    const size_t plane = (size_t)nx * ny;
    const int b = blockIdx.x;
    if (b < g.nblk_tiles) {
        int bx, by, bz;
        if (tile_of_block(g, b, bx, by, bz)) {
            const int i = 1 + bx * TX + tx, j = 1 + by * TY + ty;
            if (i <= nx - 2 && j <= ny - 2) {
                const int k0 = 1 + bz * g.TZ;
                const int k1 = min(k0 + g.TZ, g.nz - 1);
                size_t e = (size_t)i + (size_t)nx * j + (size_t)k0 * plane;
                for (int k = k0; k < k1; ++k, e += plane) {
                    if (skip_bit(skip, g, i, j, k)) continue;
                    T rv = r[e];
                    r0[e] = rv;
                    p[e] = T(0);
                    v[e] = T(0);
                    acc[0] += (double)rv * (double)rv;
                }
            }
        }
    } else {
        const int row = (b - g.nblk_tiles) * NT + tid;
        if (row < ir.n) {
            const int e = ir.node[row];
            T rv = r[e];
            r0[e] = rv;
            p[e] = T(0);
            v[e] = T(0);
            acc[0] += (double)rv * (double)rv;
        }
    }
    if (publish_partials<1>(acc, partials, ticket, nblocks)) {
        double tot[1];
        total_partials<1>(tot, partials, ticket, nblocks);
        if (tid == 0) {
            st->rho = tot[0];
            st->r0n2 = tot[0];
            st->alpha = 0.0;
            st->beta = 0.0;
            st->omega = 1.0;
            st->rn2s = st->res2s;
            st->done = (tot[0] == tot[0]) ? ((st->res2s <= st->stop2) ? 1 : 0) : 3;
        }
    }
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

template <typename T, typename TO>
void launch_apply(int mode, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *x, TO *y, const T *w,
                  const double *bvec, DevState *st)
{
    int irr_blocks = (ir.n + (NT / IRR_LANES) - 1) / (NT / IRR_LANES);
    int nb = L.g.nblk_tiles + irr_blocks;
    dim3 grid(nb), blk = tile_block();
    switch (mode) {
    case MODE_PLAIN:
        k_apply<T, TO, MODE_PLAIN><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        break;
    case MODE_V:
        k_apply<T, TO, MODE_V><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        break;
    case MODE_T:
        k_apply<T, TO, MODE_T><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        break;
    case MODE_RES:
        k_apply<T, TO, MODE_RES><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, x, y, w, bvec, st, L.partials, L.ticket, nb);
        break;
    }
}

static inline int rows_blocks(int n) { return (n + NT - 1) / NT; }

template <typename T>
void launch_cheb(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *xc, const T *xm1, const T *rho, T *xn,
                 double c1, double c2, const DevState *st)
{
    dim3 grid(L.g.nblk_tiles + rows_blocks(ir.n)), blk = tile_block();
    if (xm1 == nullptr)
        k_cheb<T, true><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st);
    else
        k_cheb<T, false><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, xc, xm1, rho, xn, (T)c1, (T)c2, st);
}

template <typename T>
void launch_first(int kind, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *r, T *ps, const T *v, T *x1,
                  double c2, const DevState *st)
{
    dim3 grid(L.g.nblk_tiles + rows_blocks(ir.n)), blk = tile_block();
    if (kind == FIRST_P)
        k_first<T, FIRST_P><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, r, ps, v, x1, (T)c2, st);
    else
        k_first<T, FIRST_S><<<grid, blk, 0, L.stream>>>(L.g, cf, ir, L.skip, r, ps, v, x1, (T)c2, st);
}

template <typename T, typename TX_>
void launch_update(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, TX_ *xs, const T *ph, const T *sh, const T *s,
                   const T *t, const T *r0, T *r, DevState *st)
{
    int nb = L.g.nblk_tiles + rows_blocks(ir.n);
    k_update<T, TX_><<<dim3(nb), tile_block(), 0, L.stream>>>(L.g, cf, ir, L.skip, xs, ph, sh, s, t, r0, r, st,
                                                              L.partials, L.ticket, nb);
}

template <typename T>
void launch_restart(const Launch &L, const Irr<T> &ir, const T *r, T *r0, T *p, T *v, DevState *st)
{
    int nb = L.g.nblk_tiles + rows_blocks(ir.n);
    k_restart<T><<<dim3(nb), tile_block(), 0, L.stream>>>(L.g, ir, L.skip, r, r0, p, v, st, L.partials, L.ticket, nb);
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
