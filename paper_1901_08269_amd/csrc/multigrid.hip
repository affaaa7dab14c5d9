// multigrid.hip -- grid transfers of the multigrid preconditioner for K.
//
// The paper preconditions BiCGSTAB with the second-order operator K (Sec. 3.3) applied
// approximately by an inner solver, and allows other inner solvers than its own.  The
// multigrid inner solver is one V-cycle on a hierarchy of grids: a coarser grid keeps, along
// every axis, the even-indexed points and the last one, and carries its own K built from the
// level set at its nodes.  Prolongation P is the tensor product of 1D linear interpolation
// in the physical coordinate; restriction is P^T with every coarse row divided by its sum.
// Both act on unknown nodes only: every other node holds 0 on every level.
//
// 1D tables per axis (built on the host from the coordinates):
//   prolongation  for each fine index i: the left coarse index a[i] and the weight w[i] of
//                 coarse node a[i] + 1 (fine value = (1 - w) e[a] + w e[a + 1])
//   restriction   for each coarse index I: three fine indices ri[3I + q] and their weights
//                 rw[3I + q], already divided by the row sum (absent entries have weight 0)
#include <hip/hip_runtime.h>

#include "cps_kernels.h"

namespace cps {

namespace {

__device__ __forceinline__ bool unknown(int8_t t) { return t == 1 || t == 2; }

// coarse rho(I, J, K) = sum over the 3 x 3 x 3 fine nodes of rwx rwy rwz r at unknown
// coarse nodes, 0 elsewhere (every coarse node is written)
template <typename T>
__global__ void k_mg_restrict(int ncx, int ncy, int ncz, int nfx, int nfy, MgAxis<T> ax, MgAxis<T> ay, MgAxis<T> az,
                              const int8_t *__restrict__ type_c, const T *__restrict__ r, T *__restrict__ rc)
{
    const int I = (int)(blockIdx.x * blockDim.x + threadIdx.x), J = (int)blockIdx.y, K = (int)blockIdx.z;
    if (I >= ncx) return;
    const size_t ec = (size_t)I + (size_t)ncx * (J + (size_t)ncy * K);
    T acc = T(0);
    if (unknown(type_c[ec])) {
        const size_t fplane = (size_t)nfx * nfy;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T wz = az.rw[3 * K + c];
            const size_t kz = (size_t)az.ri[3 * K + c] * fplane;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T wyz = wz * ay.rw[3 * J + b];
                const size_t jy = kz + (size_t)ay.ri[3 * J + b] * nfx;
                T sx = T(0);
#pragma unroll
                for (int a = 0; a < 3; ++a) sx += ax.rw[3 * I + a] * r[jy + ax.ri[3 * I + a]];
                acc += wyz * sx;
            }
        }
    }
    rc[ec] = acc;
}

// x(i, j, k) += (P e)(i, j, k) at unknown fine nodes
template <typename T>
__global__ void k_mg_prolong_add(int nfx, int nfy, int nfz, int ncx, int ncy, MgAxis<T> ax, MgAxis<T> ay,
                                 MgAxis<T> az, const int8_t *__restrict__ type_f, const T *__restrict__ e,
                                 T *__restrict__ x)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x), j = (int)blockIdx.y, k = (int)blockIdx.z;
    if (i >= nfx) return;
    const size_t ef = (size_t)i + (size_t)nfx * (j + (size_t)nfy * k);
    if (!unknown(type_f[ef])) return;
    const int a = ax.pa[i], b = ay.pa[j], c = az.pa[k];
    const T wx = ax.pw[i], wy = ay.pw[j], wz = az.pw[k];
    const size_t cplane = (size_t)ncx * ncy;
    const T *e0 = e + (size_t)c * cplane + (size_t)b * ncx + a;   // (a, b, c)
    const T *e1 = e0 + cplane;                                     // (a, b, c + 1)
    const T lo = (T(1) - wy) * ((T(1) - wx) * e0[0] + wx * e0[1]) + wy * ((T(1) - wx) * e0[ncx] + wx * e0[ncx + 1]);
    const T hi = (T(1) - wy) * ((T(1) - wx) * e1[0] + wx * e1[1]) + wy * ((T(1) - wx) * e1[ncx] + wx * e1[ncx + 1]);
    x[ef] += (T(1) - wz) * lo + wz * hi;
}

}  // namespace

template <typename T>
void launch_mg_restrict(hipStream_t s, const MgTransfer<T> &t, const int8_t *type_c, const T *r, T *rc)
{
    dim3 grid((unsigned)((t.nc[0] + 63) / 64), (unsigned)t.nc[1], (unsigned)t.nc[2]);
    k_mg_restrict<T><<<grid, 64, 0, s>>>(t.nc[0], t.nc[1], t.nc[2], t.nf[0], t.nf[1], t.ax[0], t.ax[1], t.ax[2],
                                         type_c, r, rc);
}

template <typename T>
void launch_mg_prolong_add(hipStream_t s, const MgTransfer<T> &t, const int8_t *type_f, const T *e, T *x)
{
    dim3 grid((unsigned)((t.nf[0] + 63) / 64), (unsigned)t.nf[1], (unsigned)t.nf[2]);
    k_mg_prolong_add<T><<<grid, 64, 0, s>>>(t.nf[0], t.nf[1], t.nf[2], t.nc[0], t.nc[1], t.ax[0], t.ax[1], t.ax[2],
                                            type_f, e, x);
}

template void launch_mg_restrict<double>(hipStream_t, const MgTransfer<double> &, const int8_t *, const double *,
                                         double *);
template void launch_mg_restrict<float>(hipStream_t, const MgTransfer<float> &, const int8_t *, const float *, float *);
template void launch_mg_prolong_add<double>(hipStream_t, const MgTransfer<double> &, const int8_t *, const double *,
                                            double *);
template void launch_mg_prolong_add<float>(hipStream_t, const MgTransfer<float> &, const int8_t *, const float *,
                                           float *);

}  // namespace cps
