// cps_kernels.h -- launchers of the solver's HIP kernels (host-callable).
#pragma once
#include <algorithm>

#include "cps_device.h"

namespace cps {

enum { MODE_PLAIN = 0, MODE_V = 1, MODE_T = 2, MODE_RES = 3 };
enum { FIRST_P = 0, FIRST_S = 1 };
enum { FIN_V = 0, FIN_T = 1, FIN_UPDATE = 2, FIN_RES = 3, FIN_RESTART = 4 };

struct Launch {
    Geom g;
    hipStream_t stream;
    const uint32_t *skip;
    double *partials;   // >= 2 doubles per block of the largest launch
};

// sweeps.hip
template <typename T, typename TO>
void launch_apply(int mode, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *x, TO *y, const T *w,
                  const double *bvec, DevState *st);
// rev: march down in z (consecutive sweeps alternate, see k_cheb4).  ev0/ev1 (optional, used
// on a grid whose rows fill a wavefront): events that the launch itself stamps with the
// kernel's start and end (hipExtLaunchKernelGGL)
template <typename T>
void launch_cheb(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *xc, const T *xm1, const T *rho, T *xn,
                 double c1, double c2, const DevState *st, int rev, hipEvent_t ev0 = nullptr,
                 hipEvent_t ev1 = nullptr);
// r = rho - K x at the unknown nodes (r is written there only)
template <typename T>
void launch_resid(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *x, const T *rho, T *r,
                  const DevState *st, int rev);
// r = rho - K x at the irregular nodes only (one thread per irregular row)
template <typename T>
void launch_resid_irregular(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *x, const T *rho, T *r,
                            const DevState *st);
template <typename T>
void launch_first(int kind, const Launch &L, const Coef<T> &cf, const Irr<T> &ir, const T *r, T *ps, const T *v, T *x1,
                  double c2, const DevState *st);
template <typename T, typename TX_>
void launch_update(const Launch &L, const Coef<T> &cf, const Irr<T> &ir, TX_ *xs, const T *ph, const T *sh, const T *s,
                   const T *t, const T *r0, T *r, DevState *st);
template <typename T>
void launch_restart(const Launch &L, const Irr<T> &ir, const T *r, T *r0, T *p, T *v, DevState *st);
void launch_add_correction(hipStream_t s, size_t n, double *u, const float *d);
template <typename T>
void launch_fill(hipStream_t s, size_t n, T *a, T val);
// up to 12 vectors of one grid
template <typename T>
struct VecList {
    T *p[12];
    int n;
};
// v.p[q][e] = 0 at the nodes e < nn that are not unknowns (type 1 or 2) and at e = nn ..
// nn + pad - 1, for every vector of the list; the unknowns' entries are not touched
template <typename T>
void launch_zero_off_unknowns(hipStream_t s, size_t nn, size_t pad, const int8_t *type, const VecList<T> &v);
template <typename TI, typename TO>
void launch_masked_copy(hipStream_t s, size_t n, const int8_t *type, const TI *src, TO *dst);
void launch_output(hipStream_t s, size_t n, const int8_t *type, const double *x, const double *gv, double *u);
void launch_check_finite(hipStream_t s, size_t n, const int8_t *type, const double *x, int *flag);
constexpr int DOT_BLOCKS = 1024;
// partials[2 b], partials[2 b + 1]: block b's sums of a.b and b.b over the unknown nodes
void launch_dot2_unknowns(hipStream_t s, size_t n, const int8_t *type, const double *a, const double *b,
                          double *partials);
void launch_scale(hipStream_t s, size_t n, double *x, double alpha);

// multigrid.hip: 1D transfer tables of one axis between a level and the next coarser one
template <typename T>
struct MgAxis {
    const T *pw;     // fine index i -> weight of coarse node min(i / 2, nc - 2) + 1 (prolongation)
    const T *rw;     // interior coarse index I -> weights rw[3I + q] of fine points 2I - 1 + q
                     // (restriction), divided by the row sum
};
template <typename T>
struct MgTransfer {
    int nf[3], nc[3];
    MgAxis<T> ax[3];
};
// What the restriction writes besides rho on a coarse level: diag, the diagonal of the
// level's K at its unknown nodes and 0 at every other node (it marks the unknowns), and,
// with x1 non-null, the level's first Chebyshev step from zero, x1 = c2 rc / diag K, at its
// unknown nodes.
template <typename T>
struct MgFirst {
    T *x1;
    T c2;
    const T *diag;
};
// rc = R r at the unknown coarse interior nodes (first.diag non-zero), 0 at the other
// interior nodes
template <typename T>
void launch_mg_restrict(hipStream_t s, const MgTransfer<T> &t, const T *r, T *rc, const MgFirst<T> &first);
// diag = the diagonal of K at the unknown nodes of a level (1D tables cf, or the stored row
// of an irregular node), 0 at its other nodes
template <typename T>
void launch_mg_diag(hipStream_t s, int nx, int ny, int nz, const Coef<T> &cf, const int8_t *type, const int *irr_map,
                    const T *k7, T *diag);
// rc = R (rho - K x) from the problem's grid (geometry g, skip bits, tables cf) into the
// first coarse level, the fine residual never stored: ri holds the residual at the
// irregular nodes (launch_resid_irregular) and 0 at the solid ones.  first: as for
// launch_mg_restrict.
template <typename T>
void launch_mg_resid_restrict(hipStream_t s, const Geom &g, const Coef<T> &cf, const uint32_t *skip, const T *x,
                              const T *rho, const T *ri, const MgTransfer<T> &t, T *rc, const MgFirst<T> &first,
                              const DevState *st);
// The coarsest level's `steps` Chebyshev steps (coefficients c1, c2) from 0 in one workgroup
// of MG_LDS_THREADS threads; the level has at most MG_LDS_NODES interior nodes and steps is at
// most MG_MAX_COARSE_STEPS.  irr_map: irregular row of each irregular node.  Writes out at
// the unknown nodes.
constexpr int MG_LDS_NODES = 4096;
constexpr int MG_LDS_THREADS = 1024;
constexpr int MG_MAX_COARSE_STEPS = 64;
template <typename T>
void launch_mg_coarsest(hipStream_t s, int nx, int ny, int nz, const Coef<T> &cf, const int8_t *type,
                        const int *irr_map, const T *k7, const T *rho, T *out, int steps, const T *c1, const T *c2,
                        const DevState *st);
// Several Chebyshev-Jacobi steps on a coarse level in one launch (temporal blocking): each
// workgroup owns an MG_TB_TS^3 tile of interior nodes, loads the tile and MG_TB_H layers
// around it into LDS and runs the steps there, recomputing the layers around the tile (the
// outermost layer's values go stale one layer per step, never reaching the tile).  Steps
// S.c1[s], S.c2[s], s < S.n <= MG_TB_H (one fewer with a residual), from x = xin with x_{-1}
// = 0 (the step before is either the level's first step from 0, or the first step of a pass,
// whose c1 is 0).  Writes x at the unknown nodes of xout (!= xin) and, with rout, r = rho - K x
// there.
constexpr int MG_TB_TS = 8;
constexpr int MG_TB_H = 4;
constexpr int MG_TB_THREADS = 1024;
// coarse levels with at most this many interior points smooth with temporal blocking
constexpr long long MG_TB_MAX_POINTS = 300000;
template <typename T>
struct MgSteps {
    int n;
    T c1[MG_TB_H], c2[MG_TB_H];
};
// tr, e_add: start from x + P e at the regular unknowns (e: the next coarser level's
// correction, tr: the transfers to it) instead of x.  tr, rc, first: instead of the residual
// (rout null), its restriction into that level (rho in rc, its first step as in
// launch_mg_restrict); needs S.n <= MG_TB_H - 2.
template <typename T>
void launch_mg_smooth_tb(hipStream_t s, int nx, int ny, int nz, const Coef<T> &cf, const int8_t *type,
                         const int *irr_map, const T *k7, const T *rho, const T *xin, T *xout, T *rout,
                         const MgSteps<T> &S, const DevState *st, const MgTransfer<T> *tr = nullptr,
                         const T *e_add = nullptr, T *rc = nullptr, const MgFirst<T> *first = nullptr);
// map[nodes[r]] = r for the nirr irregular rows
void launch_mg_irr_map(hipStream_t s, int nirr, const int *nodes, int *map);
// x += P e at the regular unknown fine nodes (interior nodes without a skip bit in skip_f,
// W words per x-line)
template <typename T>
void launch_mg_prolong_add(hipStream_t s, const MgTransfer<T> &t, const uint32_t *skip_f, int W, const T *e, T *x);

// sip.hip: the strongly implicit procedure for K (factors per node: b, c, d, e, f, g, h, 0)
void launch_sip_factor(hipStream_t st, int nx, int ny, int nz, const Coef<double> &cf, const int8_t *type,
                       const int *irr_map, const double *k7, double alpha, double *F, float *F32);
// one iteration: L v = r, U delta = v (delta over v), phi = delta (first) or phi += delta
template <typename T>
void launch_sip_iteration(hipStream_t st, int nx, int ny, int nz, const int8_t *type, const T *F, const T *r, T *v,
                          T *phi, int first, const DevState *dst);

// setup.hip
struct SetupOut {
    int n_irr;
    long long n_solid, n_unknown, nnz, fallback;
    double min_hb;
};

// 1D tables (FP64) from coordinates; t holds the three coordinate arrays
// the 1D tables of all three axes (8 values per index; FP64 and FP32, 3 * 8 * nmax each)
void launch_coef(hipStream_t s, int nx, int ny, int nz, int nmax, const double *xyz, double *coef, float *coef32);
// classify nodes; flags: bit0 invalid input (NaN/Inf), bit1 a wall node inside a body has a
// fluid neighbour; with phi_out, g_out and f_out non-null the fields are also copied there
void launch_classify(hipStream_t s, int nx, int ny, int nz, const double *phi, const double *g, const double *f,
                     int8_t *type, int *flags, double *phi_out = nullptr, double *g_out = nullptr,
                     double *f_out = nullptr);
void launch_mark_irregular(hipStream_t s, int nx, int ny, int nz, int8_t *type);
// ordered compaction of the irregular nodes; returns the count through *count (device int)
void launch_compact(hipStream_t s, size_t n, const int8_t *type, int8_t want, int *blockcnt, int *list, int *count,
                    int nblocks);
int compact_blocks(size_t n);
void launch_skipbits(hipStream_t s, const Geom &g, const int8_t *type, uint32_t *skip);
void launch_irr_words(hipStream_t s, const Geom &g, const int8_t *type, const int *nodes, int nirr, uint32_t *bits,
                      int *wstart);
// build irregular rows in a fixed-stride scratch (cap entries per row); ibi_tab: 12 nirr
// doubles of scratch for the table of IBIs next to the irregular nodes
void launch_build_rows(hipStream_t s, int nx, int ny, int nz, const double *x, const double *y, const double *z,
                       const double *coef, const double *phi, const double *g, const double *f, const int8_t *type,
                       int nirr, const int *nodes, const uint32_t *irr_bits, const int *irr_wstart, double *ibi_tab,
                       int cap, int *ell_col, double *ell_val, int *len, double *rhs_row, double *k7, double *bdiag,
                       double *minhb, int *fallback, int *bad);
// K rows (Shortley-Weller at nodes next to the body) of the irregular nodes only
void launch_krows(hipStream_t s, int nx, int ny, int nz, const double *x, const double *y, const double *z,
                  const double *phi, const int8_t *type, int nirr, const int *nodes, double *k7);
// dst(I, J, K) = src(ix[I], iy[J], iz[K]) on a coarse grid of ncx x ncy x ncz nodes
void launch_gather3(hipStream_t s, int ncx, int ncy, int ncz, int nfx, int nfy, const int *ix, const int *iy,
                    const int *iz, const double *src, double *dst);
void launch_scan(hipStream_t s, const int *in, int *out, int n);   // exclusive scan, out[n] = total
void launch_pack_rows(hipStream_t s, int nirr, int cap, const int *ell_col, const double *ell_val, const int *len,
                      const int *ptr, int *col, double *val64, float *val32);
void launch_rhs_regular(hipStream_t s, int nx, int ny, int nz, const double *coef, const double *f, const double *g,
                        const int8_t *type, double *rhs);
void launch_scatter_rows(hipStream_t s, int nirr, const int *nodes, const double *rhs_row, double *rhs);
void launch_to_float(hipStream_t s, size_t n, const double *a, float *b);
// min of a[n] (from 1) and sum of fb[n]; part: 2 * MINR_PARTS doubles of scratch
constexpr int MINR_PARTS = 128;
void launch_min_reduce(hipStream_t s, int n, const double *a, const int *fb, double *part, double *out_min,
                       long long *out_sum);
// cnt[t] += number of nodes of type t, t = 0..3 (cnt zeroed by the caller)
void launch_type_hist(hipStream_t s, size_t n, const int8_t *type, int *cnt);
// per-block partials (||b||^2, ||D^-1 b||^2) over the unknowns, 2 * nblocks doubles
void launch_bnorms(hipStream_t s, int nx, int ny, int nz, const double *coef, const int8_t *type, const double *b,
                   int nirr, const int *nodes, const double *bdiag, double *partials, int nblocks);

}  // namespace cps
