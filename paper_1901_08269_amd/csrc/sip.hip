// sip.hip -- the strongly implicit procedure for K phi = rho (the preconditioner option
// CPS_PRECOND_SIP).
//
// The paper solves its preconditioned system K phi = rho (Sec. 3.3) with the modified strongly
// implicit procedure of its ref. 24, whose recurrences it does not give.  This is the strongly
// implicit procedure in its original form: Stone's partial-cancellation incomplete
// factorisation M = L U of the 7-point K, extended to three dimensions.  Unknowns are ordered
// lexicographically (x fastest).  L has b, c, d at the -z, -y, -x neighbours (B, S, W) and e
// on the diagonal; U has a unit diagonal and f, g, h at the +x, +y, +z neighbours (E, N, T).
// The six positions where L U fills in beyond K's stencil hold X1 = b f_B, X2 = b g_B,
// X3 = c f_S, X4 = c h_S, X5 = d g_W, X6 = d h_W; their unknowns are approximated by
// alpha (sum of the two stencil points minus the centre), and M equals K at K's positions:
//   b = K_B / (1 + alpha (f_B + g_B)),   c = K_S / (1 + alpha (f_S + h_S)),
//   d = K_W / (1 + alpha (g_W + h_W)),
//   e = K_P - b h_B - c g_S - d f_W + alpha (X1 + ... + X6),
//   f = (K_E - alpha (X1 + X3)) / e,   g = (K_N - alpha (X2 + X5)) / e,
//   h = (K_T - alpha (X4 + X6)) / e,
// every entry toward a node that is not an unknown being 0.  One iteration is r = rho - K phi,
// L v = r, U delta = v, phi += delta.
//
// The factorisation and both substitutions are recurrences along all three axes: node
// (i, j, k) needs its -x, -y, -z neighbours first (the +x, +y, +z ones going back).  The nodes
// of one hyperplane i + j + k = s depend only on the hyperplane before, so each hyperplane is
// one launch over its nodes (one thread per (j, k) with i = s - j - k); a grid of n^3 points
// takes 3 (n - 2) - 2 launches per substitution.  This is inherently sequential work (the
// paper's inner solver is too): the library's default inner solvers are the parallel ones.
#include <hip/hip_runtime.h>

#include "cps_kernels.h"

namespace cps {

namespace {

__device__ __forceinline__ bool unk(int8_t t) { return t == 1 || t == 2; }

struct Plane {
    int s, klo;
};

// the node of hyperplane s handled by this thread, or -1
__device__ __forceinline__ long long plane_node(int nx, int ny, const Plane &p, int &i, int &j, int &k)
{
    j = 1 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    k = p.klo + (int)blockIdx.y;
    i = p.s - j - k;
    if (j > ny - 2 || i < 1 || i > nx - 2) return -1;
    return (long long)i + (long long)nx * ((long long)j + (long long)ny * k);
}

__global__ void k_sip_factor(int nx, int ny, int nz, Plane p, Coef<double> cf, const int8_t *__restrict__ type,
                             const int *__restrict__ irr_map, const double *__restrict__ k7, double alpha,
                             double *__restrict__ F, float *__restrict__ F32)
{
    int i, j, k;
    const long long e = plane_node(nx, ny, p, i, j, k);
    if (e < 0) return;
    const int8_t t = type[e];
    if (!unk(t)) return;
    const long long sy = nx, sz = (long long)nx * ny;
    double co[7];
    if (t == 2) {
        const double *r = k7 + 7 * (size_t)irr_map[e];
#pragma unroll
        for (int q = 0; q < 7; ++q) co[q] = r[q];
    } else {
        const double *cx = cf.c[0] + 8 * i, *cy = cf.c[1] + 8 * j, *cz = cf.c[2] + 8 * k;
        co[0] = (cx[6] + cy[6]) + cz[6];
        co[1] = unk(type[e - 1]) ? cx[5] : 0.0;
        co[2] = unk(type[e + 1]) ? cx[7] : 0.0;
        co[3] = unk(type[e - sy]) ? cy[5] : 0.0;
        co[4] = unk(type[e + sy]) ? cy[7] : 0.0;
        co[5] = unk(type[e - sz]) ? cz[5] : 0.0;
        co[6] = unk(type[e + sz]) ? cz[7] : 0.0;
    }
    // factors of the -z, -y, -x neighbours (zero at nodes that are not unknowns)
    const double *FB = F + 8 * (e - sz), *FS = F + 8 * (e - sy), *FW = F + 8 * (e - 1);
    const double b = co[5] / (1.0 + alpha * (FB[4] + FB[5]));
    const double c = co[3] / (1.0 + alpha * (FS[4] + FS[6]));
    const double d = co[1] / (1.0 + alpha * (FW[5] + FW[6]));
    const double X1 = b * FB[4], X2 = b * FB[5], X3 = c * FS[4], X4 = c * FS[6], X5 = d * FW[5], X6 = d * FW[6];
    const double ee = co[0] - b * FB[6] - c * FS[5] - d * FW[4] + alpha * (X1 + X2 + X3 + X4 + X5 + X6);
    double out[8];
    out[0] = b;
    out[1] = c;
    out[2] = d;
    out[3] = ee;
    out[4] = unk(type[e + 1]) ? (co[2] - alpha * (X1 + X3)) / ee : 0.0;
    out[5] = unk(type[e + sy]) ? (co[4] - alpha * (X2 + X5)) / ee : 0.0;
    out[6] = unk(type[e + sz]) ? (co[6] - alpha * (X4 + X6)) / ee : 0.0;
    out[7] = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        F[8 * e + q] = out[q];
        F32[8 * e + q] = (float)out[q];
    }
}

// L v = r on hyperplane s: v = (r - b v_B - c v_S - d v_W) / e
template <typename T>
__global__ void k_sip_fwd(int nx, int ny, Plane p, const int8_t *__restrict__ type, const T *__restrict__ F,
                          const T *__restrict__ r, T *__restrict__ v, const DevState *st)
{
    if (st && st->done) return;
    int i, j, k;
    const long long e = plane_node(nx, ny, p, i, j, k);
    if (e < 0 || !unk(type[e])) return;
    const long long sy = nx, sz = (long long)nx * ny;
    const T *f = F + 8 * e;
    v[e] = (r[e] - f[0] * v[e - sz] - f[1] * v[e - sy] - f[2] * v[e - 1]) / f[3];
}

// U delta = v on hyperplane s (delta over v): delta = v - f delta_E - g delta_N - h delta_T;
// phi = delta (first iteration) or phi += delta
template <typename T>
__global__ void k_sip_bwd(int nx, int ny, Plane p, const int8_t *__restrict__ type, const T *__restrict__ F,
                          T *__restrict__ v, T *__restrict__ phi, int first, const DevState *st)
{
    if (st && st->done) return;
    int i, j, k;
    const long long e = plane_node(nx, ny, p, i, j, k);
    if (e < 0 || !unk(type[e])) return;
    const long long sy = nx, sz = (long long)nx * ny;
    const T *f = F + 8 * e;
    const T dl = v[e] - (f[4] * v[e + 1] + f[5] * v[e + sy] + f[6] * v[e + sz]);
    v[e] = dl;
    phi[e] = first ? dl : phi[e] + dl;
}

// launch shape of hyperplane s: threads over j, blocks over the k that reach it
inline bool plane_launch(int nx, int ny, int nz, int s, Plane &p, dim3 &grid)
{
    const int klo = std::max(1, s - (nx - 2) - (ny - 2)), khi = std::min(nz - 2, s - 2);
    if (khi < klo) return false;
    p.s = s;
    p.klo = klo;
    grid = dim3((unsigned)((ny - 2 + 255) / 256), (unsigned)(khi - klo + 1));
    return true;
}

}  // namespace

void launch_sip_factor(hipStream_t st, int nx, int ny, int nz, const Coef<double> &cf, const int8_t *type,
                       const int *irr_map, const double *k7, double alpha, double *F, float *F32)
{
    for (int s = 3; s <= (nx - 2) + (ny - 2) + (nz - 2); ++s) {
        Plane p;
        dim3 grid;
        if (plane_launch(nx, ny, nz, s, p, grid))
            k_sip_factor<<<grid, 256, 0, st>>>(nx, ny, nz, p, cf, type, irr_map, k7, alpha, F, F32);
    }
}

template <typename T>
void launch_sip_iteration(hipStream_t st, int nx, int ny, int nz, const int8_t *type, const T *F, const T *r, T *v,
                          T *phi, int first, const DevState *dst)
{
    const int smax = (nx - 2) + (ny - 2) + (nz - 2);
    for (int s = 3; s <= smax; ++s) {
        Plane p;
        dim3 grid;
        if (plane_launch(nx, ny, nz, s, p, grid)) k_sip_fwd<T><<<grid, 256, 0, st>>>(nx, ny, p, type, F, r, v, dst);
    }
    for (int s = smax; s >= 3; --s) {
        Plane p;
        dim3 grid;
        if (plane_launch(nx, ny, nz, s, p, grid))
            k_sip_bwd<T><<<grid, 256, 0, st>>>(nx, ny, p, type, F, v, phi, first, dst);
    }
}

template void launch_sip_iteration<double>(hipStream_t, int, int, int, const int8_t *, const double *, const double *,
                                           double *, double *, int, const DevState *);
template void launch_sip_iteration<float>(hipStream_t, int, int, int, const int8_t *, const float *, const float *,
                                          float *, float *, int, const DevState *);

}  // namespace cps
