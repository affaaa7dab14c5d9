/*
 * cps_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU reference for the fourth-order compact immersed-interface
 * discretisation of the 3D Dirichlet Poisson problem (Hosseinverdi & Fasel, arXiv
 * 1901.08269) and for its right-preconditioned BiCGSTAB solve.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load this library; the GPU
 * library shares no code, header or table with it.
 *
 * Conventions
 *   node (i,j,k) <-> flat index i + nx*(j + ny*k); 0-based, boundary planes included.
 *   node type: 0 boundary (value g), 1 regular fluid, 2 irregular fluid, 3 solid (value 0).
 *   every vector is a full-grid array; only unknown (fluid) entries are meaningful.
 *
 * Readings of the paper taken here (ambiguities and silences):
 *   - IBIs exist only where the nodal level set changes sign between adjacent nodes; the
 *     IBI is the root of the degree-5 Lagrange interpolant of nodal phi through six nodes
 *     straddling the segment (window shifted to stay inside the grid), found by bisection;
 *     the Dirichlet value there is the same interpolant applied to nodal g.
 *   - One-sided operators (Sec. 2.2, Eqs. mod1-mod4 / mat1-mat4; Sec. 2.3, Eqs.
 *     mod2_case2 / mod2_case22) are computed from polynomial exactness: the weights on the
 *     point set P reproduce sum_{p in run} L[p] u''(x_p) exactly for every polynomial of
 *     degree < |P|.  This is the Taylor-matching system M of Eq. (M) written in moments.
 *     |P| = 6 for a window with one fluid run next to one IBI, 5 for each run of an F-S-F
 *     window; an S-F-S window uses {IBI, node, IBI}.  When the march for extra points meets
 *     a wall node it keeps that (known) node and stops; when it meets another solid node it
 *     ends at that IBI.  Each shortened or S-F-S set counts as a fallback line.
 *   - Preconditioner inner solve: the paper's MSI (ref. 24) is not reproduced; K is solved
 *     approximately by `iters` steps of Chebyshev-accelerated Jacobi from phi_0 = 0
 *     (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1), a fixed linear map.
 *   - Stopping (the paper gives none): the recursive Jacobi-weighted residual
 *     ||D^{-1} r||_2 / ||D^{-1} b||_2 <= tol (D = diag B), confirmed on the true residual
 *     together with ||r||_2 / ||b||_2 <= tol in the paper's own row scaling.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;

enum { T_BOUND = 0, T_REG = 1, T_IRR = 2, T_SOLID = 3 };

typedef struct {
    int n[3];          /* points per direction: nx, ny, nz */
    i64 stride[3];     /* 1, nx, nx*ny */
    i64 nn;            /* total nodes */
    double *t[3];      /* coordinates */
    double *phi, *g, *f;
    signed char *type;
    /* compact coefficients per direction and index: L = (a, 1, c), R = (ar, br, cr) */
    double *La[3], *Lc[3], *Ra[3], *Rb[3], *Rc[3];
    /* second-order coefficients (Eq. 2ndorder_coef) */
    double *Ka[3], *Kb[3], *Kc[3];
    /* irregular rows of B, CSR over node indices (unknown columns only) */
    i64 nirr;
    i64 *irr_node, *irr_ptr, *irr_col;
    double *irr_val;
    i64 *irr_of_node;  /* node -> irregular row, -1 otherwise */
    double *ksw;       /* per irregular row: K row [diag, -x, +x, -y, +y, -z, +z] */
    double *rhs;       /* right-hand side of B u = q + b at unknown nodes */
    i64 n_unknown, n_solid, fallback;
    double min_hb;     /* min over IBIs of (distance fluid node -> IBI) / segment length */
} orc_prob;

/* ------------------------------------------------------------------------------------ */
/* 1D coefficients                                                                      */
/* ------------------------------------------------------------------------------------ */

/* Eq. (app_xxx): fourth-order compact relation a u''_{i-1} + u''_i + c u''_{i+1}
 * = ar u_{i-1} + br u_i + cr u_{i+1} with dx_f = x_{i+1}-x_i, dx_b = x_i-x_{i-1}. */
void orc_compact_coef(int n, const double *x, double *a, double *c, double *ar, double *br, double *cr)
{
    for (int i = 0; i < n; ++i) {
        a[i] = c[i] = ar[i] = br[i] = cr[i] = 0.0;
        if (i == 0 || i == n - 1) continue;
        double f = x[i + 1] - x[i], b = x[i] - x[i - 1];
        double den = f * f * f + 4.0 * f * f * b + 4.0 * f * b * b + b * b * b;
        a[i] = f * (b * b + b * f - f * f) / den;
        c[i] = b * (f * f + b * f - b * b) / den;
        ar[i] = 12.0 * f / den;
        br[i] = -12.0 / (f * f + 3.0 * f * b + b * b);
        cr[i] = 12.0 * b / den;
    }
}

/* Eq. (2ndorder_coef): three-point second derivative on a nonuniform grid. */
static void sw_coef(double dxb, double dxf, double *a, double *b, double *c)
{
    *a = 2.0 / (dxb * (dxf + dxb));
    *b = -2.0 / (dxb * dxf);
    *c = 2.0 / (dxf * (dxf + dxb));
}

void orc_second_coef(int n, const double *x, double *a, double *b, double *c)
{
    for (int i = 0; i < n; ++i) {
        a[i] = b[i] = c[i] = 0.0;
        if (i == 0 || i == n - 1) continue;
        sw_coef(x[i] - x[i - 1], x[i + 1] - x[i], &a[i], &b[i], &c[i]);
    }
}

/* ------------------------------------------------------------------------------------ */
/* geometry helpers                                                                     */
/* ------------------------------------------------------------------------------------ */

static i64 nid(const orc_prob *P, int i, int j, int k) { return i + (i64)P->n[0] * (j + (i64)P->n[1] * k); }

static void coords_of(const orc_prob *P, i64 node, int c[3])
{
    c[0] = (int)(node % P->n[0]);
    c[1] = (int)((node / P->n[0]) % P->n[1]);
    c[2] = (int)(node / ((i64)P->n[0] * P->n[1]));
}

static int is_solid(const orc_prob *P, i64 node) { return P->type[node] == T_SOLID; }
static int is_unknown(const orc_prob *P, i64 node) { return P->type[node] == T_REG || P->type[node] == T_IRR; }

/* value of the degree-(m-1) Lagrange interpolant through (ts[s], vs[s]) at t */
static double lagrange(int m, const double *ts, const double *vs, double t)
{
    double sum = 0.0;
    for (int s = 0; s < m; ++s) {
        double w = 1.0;
        for (int q = 0; q < m; ++q)
            if (q != s) w *= (t - ts[q]) / (ts[s] - ts[q]);
        sum += w * vs[s];
    }
    return sum;
}

/* Immersed-boundary intersection on the grid segment between the fluid node `ia` and the
 * solid node `ib` (= ia +- 1) of the grid line along direction d through node `line0`
 * (the line's node with index 0 along d).  Returns the IBI coordinate; *gv = g there. */
static double ibi_point(orc_prob *P, int d, i64 line0, int ia, int ib, double *gv)
{
    int n = P->n[d];
    int m = ia < ib ? ia : ib;
    int cnt = n < 6 ? n : 6;
    int s0 = m - 2;
    if (s0 > n - cnt) s0 = n - cnt;
    if (s0 < 0) s0 = 0;
    double ts[6], ph[6], gs[6];
    for (int s = 0; s < cnt; ++s) {
        i64 node = line0 + (i64)(s0 + s) * P->stride[d];
        ts[s] = P->t[d][s0 + s];
        ph[s] = P->phi[node];
        gs[s] = P->g[node];
    }
    double ta = P->t[d][ia], tb = P->t[d][ib];
    double root;
    double phb = P->phi[line0 + (i64)ib * P->stride[d]];
    if (phb == 0.0) {
        root = tb;
    } else {
        /* bisection keeping lagrange(fluid end) > 0 >= lagrange(solid end) */
        double lo = ta, hi = tb;
        for (int it = 0; it < 200; ++it) {
            double mid = lo + 0.5 * (hi - lo);
            if (mid == lo || mid == hi) break;
            double v = lagrange(cnt, ts, ph, mid);
            if (v > 0.0) lo = mid; else hi = mid;
        }
        root = lo + 0.5 * (hi - lo);
    }
    double frac = fabs(root - ta) / fabs(tb - ta);
    if (frac < P->min_hb) P->min_hb = frac;
    *gv = lagrange(cnt, ts, gs, root);
    return root;
}

/* ------------------------------------------------------------------------------------ */
/* row accumulator                                                                      */
/* ------------------------------------------------------------------------------------ */
#define ROW_CAP 512
typedef struct {
    int cnt;
    i64 col[ROW_CAP];
    double val[ROW_CAP];
    double rhs;
} row_acc;

/* coefficient `v` multiplies u at `node`: unknown -> matrix entry, wall node -> moved to
 * the right-hand side with its Dirichlet value g */
static void acc_node(const orc_prob *P, row_acc *R, i64 node, double v)
{
    if (P->type[node] == T_BOUND) {
        R->rhs -= v * P->g[node];
        return;
    }
    for (int e = 0; e < R->cnt; ++e)
        if (R->col[e] == node) {
            R->val[e] += v;
            return;
        }
    if (R->cnt >= ROW_CAP) {
        fprintf(stderr, "oracle: row capacity exceeded\n");
        abort();
    }
    R->col[R->cnt] = node;
    R->val[R->cnt] = v;
    R->cnt++;
}

/* ------------------------------------------------------------------------------------ */
/* one-sided operator weights (Sec. 2.2 Eqs. mat1-mat4 and M; Sec. 2.3)                  */
/* ------------------------------------------------------------------------------------ */

/* Solve the small dense system A w = b (A is m x m, row-major) by Gaussian elimination
 * with partial pivoting.  Returns 0 on success. */
static int dense_solve(int m, double *A, double *b, double *w)
{
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[r * m + col]) > fabs(A[piv * m + col])) piv = r;
        if (A[piv * m + col] == 0.0) return -1;
        if (piv != col) {
            for (int q = 0; q < m; ++q) {
                double tmp = A[col * m + q];
                A[col * m + q] = A[piv * m + q];
                A[piv * m + q] = tmp;
            }
            double tmp = b[col];
            b[col] = b[piv];
            b[piv] = tmp;
        }
        for (int r = col + 1; r < m; ++r) {
            double fct = A[r * m + col] / A[col * m + col];
            for (int q = col; q < m; ++q) A[r * m + q] -= fct * A[col * m + q];
            b[r] -= fct * b[col];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        double s = b[r];
        for (int q = r + 1; q < m; ++q) s -= A[r * m + q] * w[q];
        w[r] = s / A[r * m + r];
    }
    return 0;
}

/* Weights w over the points tp[0..np) such that sum_pi w_pi u(tp_pi) equals
 * sum_{s<nrun} Lw[s] u''(tr[s]) for every polynomial u of degree < np.
 * tref/href scale the coordinates for conditioning only (the conditions are
 * translation invariant).  Exposed for the tests that check Eqs. (mat1)-(mat4). */
int orc_onesided_weights(int np, const double *tp, int nrun, const double *tr, const double *Lw,
                         double tref, double href, double *w)
{
    double A[64], b[8];
    if (np > 8 || np < 1) return -1;
    for (int m = 0; m < np; ++m) {
        for (int q = 0; q < np; ++q) A[m * np + q] = pow((tp[q] - tref) / href, m);
        double s = 0.0;
        if (m >= 2)
            for (int r = 0; r < nrun; ++r) s += Lw[r] * m * (m - 1) * pow((tr[r] - tref) / href, m - 2);
        b[m] = s / (href * href);
    }
    return dense_solve(np, A, b, w);
}

/* ------------------------------------------------------------------------------------ */
/* regular 27-point row: Eqs. (A27), (As_qs), (q)                                        */
/* ------------------------------------------------------------------------------------ */

/* Fill the 27 coefficients A^{9 alpha + m} and q^{9 alpha + m} of the row at (i,j,k) and
 * the offsets of the node each multiplies.  Numbering: alpha = 0,1,2 <-> z offset -1,0,+1
 * (beta = a, b, c); inside a plane m = 1..3 is y+1, 4..6 is y, 7..9 is y-1, and each
 * triple runs over x-1, x, x+1. */
static void regular_row(const orc_prob *P, int i, int j, int k, double A[27], double q[27], int off[27][3])
{
    double Lx[3] = {P->La[0][i], 1.0, P->Lc[0][i]}, Rx[3] = {P->Ra[0][i], P->Rb[0][i], P->Rc[0][i]};
    double Ly[3] = {P->La[1][j], 1.0, P->Lc[1][j]}, Ry[3] = {P->Ra[1][j], P->Rb[1][j], P->Rc[1][j]};
    double Lz[3] = {P->La[2][k], 1.0, P->Lc[2][k]}, Rz[3] = {P->Ra[2][k], P->Rb[2][k], P->Rc[2][k]};
    for (int alpha = 0; alpha < 3; ++alpha) {
        double beta = Lz[alpha], betar = Rz[alpha];
        for (int m = 1; m <= 9; ++m) {
            int px = (m - 1) % 3;          /* 0,1,2 <-> x-1, x, x+1 */
            int qy = 2 - (m - 1) / 3;      /* 2,1,0 <-> y+1, y, y-1 */
            int e = 9 * alpha + m - 1;
            A[e] = Rx[px] * Ly[qy] * beta + Lx[px] * Ry[qy] * beta + Lx[px] * Ly[qy] * betar;
            q[e] = Lx[px] * Ly[qy] * beta;
            off[e][0] = px - 1;
            off[e][1] = qy - 1;
            off[e][2] = alpha - 1;
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* irregular row: Eq. (lhsrhs_xxyyzz_mod) with the modified operators of Secs. 2.2-2.3   */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    double t;       /* coordinate along the line */
    int kind;       /* 0: grid node, 1: IBI */
    i64 node;       /* grid node (kind 0) */
    double gval;    /* Dirichlet value (kind 1) */
} pt_t;

/* One fluid run [plo, phi_] (window positions -1..1 relative to index c along direction d)
 * of a window that meets the body.  Builds the point set P, solves for the one-sided
 * weights and adds W * w into the row. */
static void modified_run(orc_prob *P, row_acc *R, int d, i64 line0, int c, int plo, int phi_,
                         const int solidpos[3], int nruns, const double Ld[3], double W)
{
    int n = P->n[d];
    pt_t pts[8];
    int np = 0;
    int left_solid = (plo > -1) && solidpos[plo - 1 + 1];
    int right_solid = (phi_ < 1) && solidpos[phi_ + 1 + 1];
    double gv;
    double tr[3], Lw[3];
    int nrun = 0;
    for (int p = plo; p <= phi_; ++p) {
        tr[nrun] = P->t[d][c + p];
        Lw[nrun] = Ld[p + 1];
        nrun++;
    }
    int fallback = 0;
    if (left_solid && right_solid) {
        /* S-F-S: {IBI-, node, IBI+} */
        double tl = ibi_point(P, d, line0, c + plo, c + plo - 1, &gv);
        pts[np++] = (pt_t){tl, 1, -1, gv};
        for (int p = plo; p <= phi_; ++p) pts[np++] = (pt_t){P->t[d][c + p], 0, line0 + (i64)(c + p) * P->stride[d], 0.0};
        double th = ibi_point(P, d, line0, c + phi_, c + phi_ + 1, &gv);
        pts[np++] = (pt_t){th, 1, -1, gv};
        fallback = 1;
    } else {
        int target = (nruns == 2) ? 5 : 6;
        int dir = right_solid ? -1 : +1;   /* march away from the interface */
        int iend_solid = right_solid ? c + phi_ : c + plo;   /* run node next to the IBI */
        int isolid = right_solid ? c + phi_ + 1 : c + plo - 1;
        for (int p = plo; p <= phi_; ++p) pts[np++] = (pt_t){P->t[d][c + p], 0, line0 + (i64)(c + p) * P->stride[d], 0.0};
        double tb = ibi_point(P, d, line0, iend_solid, isolid, &gv);
        pts[np++] = (pt_t){tb, 1, -1, gv};
        int idx = (dir < 0) ? c + plo : c + phi_;
        while (np < target) {
            int nxt = idx + dir;
            if (nxt < 0 || nxt >= n) { fallback = 1; break; }
            i64 node = line0 + (i64)nxt * P->stride[d];
            if (P->type[node] == T_SOLID) {
                double te = ibi_point(P, d, line0, idx, nxt, &gv);
                pts[np++] = (pt_t){te, 1, -1, gv};
                fallback = 1;
                break;
            }
            pts[np++] = (pt_t){P->t[d][nxt], 0, node, 0.0};
            idx = nxt;
            if (P->type[node] == T_BOUND) {
                if (np < target) fallback = 1;
                break;
            }
        }
        if (np < target) fallback = 1;
    }
    if (fallback) P->fallback++;
    /* scaling: reference = run node nearest the interface, scale = largest offset */
    double tref = right_solid ? P->t[d][c + phi_] : P->t[d][c + plo];
    double href = 0.0;
    double tp[8], w[8];
    for (int s = 0; s < np; ++s) {
        tp[s] = pts[s].t;
        if (fabs(tp[s] - tref) > href) href = fabs(tp[s] - tref);
    }
    if (orc_onesided_weights(np, tp, nrun, tr, Lw, tref, href, w) != 0) {
        fprintf(stderr, "oracle: singular one-sided system\n");
        abort();
    }
    for (int s = 0; s < np; ++s) {
        if (pts[s].kind == 0) acc_node(P, R, pts[s].node, W * w[s]);
        else R->rhs -= W * w[s] * pts[s].gval;
    }
}

static void irregular_row(orc_prob *P, int i, int j, int k, row_acc *R)
{
    int c[3] = {i, j, k};
    double L[3][3], Rr[3][3];
    for (int d = 0; d < 3; ++d) {
        L[d][0] = P->La[d][c[d]]; L[d][1] = 1.0; L[d][2] = P->Lc[d][c[d]];
        Rr[d][0] = P->Ra[d][c[d]]; Rr[d][1] = P->Rb[d][c[d]]; Rr[d][2] = P->Rc[d][c[d]];
    }
    R->cnt = 0;
    R->rhs = 0.0;
    /* Q-bar: Eq. (q) with the weights of solid nodes removed */
    for (int r = -1; r <= 1; ++r)
        for (int q = -1; q <= 1; ++q)
            for (int p = -1; p <= 1; ++p) {
                i64 node = nid(P, i + p, j + q, k + r);
                if (!is_solid(P, node)) R->rhs += L[0][p + 1] * L[1][q + 1] * L[2][r + 1] * P->f[node];
            }
    /* the 27 line windows: 9 per direction, each weighted by the row's L in the two
     * transverse directions */
    for (int d = 0; d < 3; ++d) {
        int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int s = -1; s <= 1; ++s)
            for (int t = -1; t <= 1; ++t) {
                double W = L[d1][s + 1] * L[d2][t + 1];
                int b[3] = {c[0], c[1], c[2]};
                b[d1] += s;
                b[d2] += t;
                int b0[3] = {b[0], b[1], b[2]};
                b0[d] = 0;
                i64 line0 = nid(P, b0[0], b0[1], b0[2]);
                int sol[3];
                int nsol = 0;
                for (int p = -1; p <= 1; ++p) {
                    sol[p + 1] = is_solid(P, line0 + (i64)(c[d] + p) * P->stride[d]);
                    nsol += sol[p + 1];
                }
                if (nsol == 0) {
                    for (int p = -1; p <= 1; ++p)
                        acc_node(P, R, line0 + (i64)(c[d] + p) * P->stride[d], W * Rr[d][p + 1]);
                    continue;
                }
                if (nsol == 3) continue;   /* window wholly inside the body: dropped */
                /* maximal fluid runs */
                int runs[2][2], nr = 0;
                int p = -1;
                while (p <= 1) {
                    if (sol[p + 1]) { ++p; continue; }
                    int lo = p;
                    while (p + 1 <= 1 && !sol[p + 2]) ++p;
                    runs[nr][0] = lo;
                    runs[nr][1] = p;
                    nr++;
                    ++p;
                }
                for (int e = 0; e < nr; ++e)
                    modified_run(P, R, d, line0, c[d], runs[e][0], runs[e][1], sol, nr, L[d], W);
            }
    }
}

/* ------------------------------------------------------------------------------------ */
/* setup                                                                                */
/* ------------------------------------------------------------------------------------ */

static double *dalloc(i64 n) { return (double *)calloc((size_t)n, sizeof(double)); }

void orc_destroy(void *h)
{
    orc_prob *P = (orc_prob *)h;
    if (!P) return;
    for (int d = 0; d < 3; ++d) {
        free(P->t[d]); free(P->La[d]); free(P->Lc[d]); free(P->Ra[d]); free(P->Rb[d]); free(P->Rc[d]);
        free(P->Ka[d]); free(P->Kb[d]); free(P->Kc[d]);
    }
    free(P->phi); free(P->g); free(P->f); free(P->type);
    free(P->irr_node); free(P->irr_ptr); free(P->irr_col); free(P->irr_val); free(P->irr_of_node);
    free(P->ksw); free(P->rhs);
    free(P);
}

/* K row at unknown node (i,j,k): Eq. (A7), Shortley-Weller modified at solid axis
 * neighbours (Eqs. 2ndorder_coef_mod, A7_mod).  coef = [diag, -x, +x, -y, +y, -z, +z];
 * neighbours that are wall or solid nodes get coefficient 0 (zero Dirichlet data). */
static void k_row(orc_prob *P, int i, int j, int k, double coef[7])
{
    int c[3] = {i, j, k};
    coef[0] = 0.0;
    for (int d = 0; d < 3; ++d) {
        int b0[3] = {i, j, k};
        b0[d] = 0;
        i64 line0 = nid(P, b0[0], b0[1], b0[2]);
        i64 nm = line0 + (i64)(c[d] - 1) * P->stride[d], np_ = line0 + (i64)(c[d] + 1) * P->stride[d];
        double dxb = P->t[d][c[d]] - P->t[d][c[d] - 1], dxf = P->t[d][c[d] + 1] - P->t[d][c[d]];
        double gv;
        if (is_solid(P, nm)) dxb = P->t[d][c[d]] - ibi_point(P, d, line0, c[d], c[d] - 1, &gv);
        if (is_solid(P, np_)) dxf = ibi_point(P, d, line0, c[d], c[d] + 1, &gv) - P->t[d][c[d]];
        double a, b, cc;
        sw_coef(dxb, dxf, &a, &b, &cc);
        coef[0] += b;
        coef[1 + 2 * d] = is_unknown(P, nm) ? a : 0.0;
        coef[2 + 2 * d] = is_unknown(P, np_) ? cc : 0.0;
    }
}

/* returns NULL and *err < 0 on invalid input: -1 bad sizes/coords, -2 a fluid node next to a
 * wall node that lies in a body.
 * k_only: classification and the K rows only (no rows of B, no right-hand side), for the
 * coarse levels of the multigrid preconditioner. */
static void *create(int nx, int ny, int nz, const double *x, const double *y, const double *z,
                    const double *phi, const double *g, const double *f, int k_only, int *err)
{
    *err = 0;
    if (nx < 3 || ny < 3 || nz < 3) { *err = -1; return NULL; }
    const double *co[3] = {x, y, z};
    int nn3[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i + 1 < nn3[d]; ++i)
            if (!(co[d][i + 1] > co[d][i])) { *err = -1; return NULL; }
    orc_prob *P = (orc_prob *)calloc(1, sizeof(orc_prob));
    P->n[0] = nx; P->n[1] = ny; P->n[2] = nz;
    P->stride[0] = 1; P->stride[1] = nx; P->stride[2] = (i64)nx * ny;
    P->nn = (i64)nx * ny * nz;
    P->min_hb = 1.0;
    for (int d = 0; d < 3; ++d) {
        int n = P->n[d];
        P->t[d] = dalloc(n);
        memcpy(P->t[d], co[d], sizeof(double) * n);
        P->La[d] = dalloc(n); P->Lc[d] = dalloc(n); P->Ra[d] = dalloc(n); P->Rb[d] = dalloc(n); P->Rc[d] = dalloc(n);
        P->Ka[d] = dalloc(n); P->Kb[d] = dalloc(n); P->Kc[d] = dalloc(n);
        orc_compact_coef(n, P->t[d], P->La[d], P->Lc[d], P->Ra[d], P->Rb[d], P->Rc[d]);
        orc_second_coef(n, P->t[d], P->Ka[d], P->Kb[d], P->Kc[d]);
    }
    P->phi = dalloc(P->nn); P->g = dalloc(P->nn); P->f = dalloc(P->nn);
    memcpy(P->phi, phi, sizeof(double) * P->nn);
    memcpy(P->g, g, sizeof(double) * P->nn);
    memcpy(P->f, f, sizeof(double) * P->nn);
    for (i64 e = 0; e < P->nn; ++e)
        if (!isfinite(phi[e]) || !isfinite(g[e]) || !isfinite(f[e])) { *err = -1; orc_destroy(P); return NULL; }
    /* classification (Sec. 2, Fig. grid_point_types) */
    P->type = (signed char *)calloc((size_t)P->nn, 1);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                i64 e = nid(P, i, j, k);
                int wall = (i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1);
                if (wall) {
                    /* A wall node may lie in a body (an interior problem: the fluid region is
                     * inside Gamma and the walls outside it) as long as no fluid node is among
                     * its neighbours, so that no row of the scheme reaches it.  On a coarse
                     * level of the multigrid hierarchy (k_only) this is not checked: there a
                     * wall node is a zero Dirichlet node of the correction equation. */
                    if (phi[e] <= 0.0 && !k_only) {
                        for (int r = -1; r <= 1; ++r)
                            for (int q = -1; q <= 1; ++q)
                                for (int p = -1; p <= 1; ++p) {
                                    int a = i + p, b = j + q, c = k + r;
                                    if (a < 1 || b < 1 || c < 1 || a > nx - 2 || b > ny - 2 || c > nz - 2) continue;
                                    if (phi[nid(P, a, b, c)] > 0.0) { *err = -2; orc_destroy(P); return NULL; }
                                }
                    }
                    P->type[e] = T_BOUND;
                } else {
                    P->type[e] = phi[e] <= 0.0 ? T_SOLID : T_REG;
                }
            }
    P->irr_of_node = (i64 *)malloc(sizeof(i64) * P->nn);
    for (i64 e = 0; e < P->nn; ++e) P->irr_of_node[e] = -1;
    for (int k = 1; k < nz - 1; ++k)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                i64 e = nid(P, i, j, k);
                if (P->type[e] == T_SOLID) { P->n_solid++; continue; }
                P->n_unknown++;
                int irr = 0;
                for (int r = -1; r <= 1 && !irr; ++r)
                    for (int q = -1; q <= 1 && !irr; ++q)
                        for (int p = -1; p <= 1 && !irr; ++p)
                            if (phi[nid(P, i + p, j + q, k + r)] <= 0.0 &&
                                !(i + p == 0 || j + q == 0 || k + r == 0 || i + p == nx - 1 || j + q == ny - 1 || k + r == nz - 1))
                                irr = 1;
                if (irr) { P->type[e] = T_IRR; P->irr_of_node[e] = P->nirr++; }
            }
    /* irregular rows */
    P->irr_node = (i64 *)malloc(sizeof(i64) * (P->nirr + 1));
    P->irr_ptr = (i64 *)malloc(sizeof(i64) * (P->nirr + 1));
    P->ksw = dalloc(7 * (P->nirr + 1));
    P->rhs = dalloc(P->nn);
    i64 cap = 64 * (P->nirr + 1), nnz = 0;
    P->irr_col = (i64 *)malloc(sizeof(i64) * cap);
    P->irr_val = dalloc(cap);
    row_acc *R = (row_acc *)malloc(sizeof(row_acc));
    P->irr_ptr[0] = 0;
    for (i64 e = 0; e < P->nn; ++e) {
        i64 r = P->irr_of_node[e];
        if (r < 0) continue;
        int c[3];
        coords_of(P, e, c);
        P->irr_node[r] = e;
        if (k_only) {
            P->irr_ptr[r + 1] = nnz;
            k_row(P, c[0], c[1], c[2], &P->ksw[7 * r]);
            continue;
        }
        irregular_row(P, c[0], c[1], c[2], R);
        if (nnz + R->cnt > cap) {
            cap = 2 * cap + R->cnt;
            P->irr_col = (i64 *)realloc(P->irr_col, sizeof(i64) * cap);
            P->irr_val = (double *)realloc(P->irr_val, sizeof(double) * cap);
        }
        for (int q = 0; q < R->cnt; ++q) {
            P->irr_col[nnz] = R->col[q];
            P->irr_val[nnz] = R->val[q];
            nnz++;
        }
        P->irr_ptr[r + 1] = nnz;
        P->rhs[e] = R->rhs;
        k_row(P, c[0], c[1], c[2], &P->ksw[7 * r]);
    }
    free(R);
    if (k_only) return P;
    /* regular rows: Q f minus the known wall-node terms */
    for (int k = 1; k < nz - 1; ++k)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                i64 e = nid(P, i, j, k);
                if (P->type[e] != T_REG) continue;
                double A[27], q[27];
                int off[27][3];
                regular_row(P, i, j, k, A, q, off);
                double s = 0.0;
                for (int m = 0; m < 27; ++m) {
                    i64 nb = nid(P, i + off[m][0], j + off[m][1], k + off[m][2]);
                    s += q[m] * P->f[nb];
                    if (P->type[nb] == T_BOUND) s -= A[m] * P->g[nb];
                }
                P->rhs[e] = s;
            }
    return P;
}

void *orc_create(int nx, int ny, int nz, const double *x, const double *y, const double *z,
                 const double *phi, const double *g, const double *f, int *err)
{
    return create(nx, ny, nz, x, y, z, phi, g, f, 0, err);
}

/* the grid, node types and K rows only (g = f = 0) */
void *orc_create_k(int nx, int ny, int nz, const double *x, const double *y, const double *z, const double *phi,
                   int *err)
{
    i64 nn = (i64)nx * ny * nz;
    double *zero = dalloc(nn > 0 ? nn : 1);
    void *h = create(nx, ny, nz, x, y, z, phi, zero, zero, 1, err);
    free(zero);
    return h;
}

/* ------------------------------------------------------------------------------------ */
/* introspection                                                                        */
/* ------------------------------------------------------------------------------------ */

/* out: [n_unknown, n_irregular, n_solid, fallback_lines, nnz_irregular] */
void orc_info(void *h, i64 *out)
{
    orc_prob *P = (orc_prob *)h;
    out[0] = P->n_unknown; out[1] = P->nirr; out[2] = P->n_solid; out[3] = P->fallback;
    out[4] = P->irr_ptr[P->nirr];
}

double orc_min_hb(void *h) { return ((orc_prob *)h)->min_hb; }

void orc_types(void *h, signed char *out) { orc_prob *P = (orc_prob *)h; memcpy(out, P->type, (size_t)P->nn); }

void orc_rhs(void *h, double *out) { orc_prob *P = (orc_prob *)h; memcpy(out, P->rhs, sizeof(double) * P->nn); }

void orc_irregular_nodes(void *h, i64 *out) { orc_prob *P = (orc_prob *)h; memcpy(out, P->irr_node, sizeof(i64) * P->nirr); }

/* Row of B at an unknown node: unknown columns and values (unsorted). Returns the count,
 * or -1 if the node is not an unknown. */
int orc_row(void *h, i64 node, i64 *cols, double *vals, int cap)
{
    orc_prob *P = (orc_prob *)h;
    if (node < 0 || node >= P->nn || !is_unknown(P, node)) return -1;
    if (P->type[node] == T_IRR) {
        i64 r = P->irr_of_node[node];
        int cnt = (int)(P->irr_ptr[r + 1] - P->irr_ptr[r]);
        for (int e = 0; e < cnt && e < cap; ++e) {
            cols[e] = P->irr_col[P->irr_ptr[r] + e];
            vals[e] = P->irr_val[P->irr_ptr[r] + e];
        }
        return cnt;
    }
    int c[3];
    coords_of(P, node, c);
    double A[27], q[27];
    int off[27][3];
    regular_row(P, c[0], c[1], c[2], A, q, off);
    int cnt = 0;
    for (int m = 0; m < 27; ++m) {
        i64 nb = nid(P, c[0] + off[m][0], c[1] + off[m][1], c[2] + off[m][2]);
        if (!is_unknown(P, nb)) continue;
        if (cnt < cap) { cols[cnt] = nb; vals[cnt] = A[m]; }
        cnt++;
    }
    return cnt;
}

/* K row at an unknown node: coefficient order [diag, -x, +x, -y, +y, -z, +z] */
int orc_krow(void *h, i64 node, double *coef)
{
    orc_prob *P = (orc_prob *)h;
    if (node < 0 || node >= P->nn || !is_unknown(P, node)) return -1;
    int c[3];
    coords_of(P, node, c);
    k_row(P, c[0], c[1], c[2], coef);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* operators                                                                            */
/* ------------------------------------------------------------------------------------ */

/* y = B x at every unknown node (Eq. Bu=q with B = A-bar + C, Eq. Bdec); y = 0 elsewhere.
 * Entries of x at non-unknown nodes are ignored. */
void orc_apply(void *h, const double *x, double *y)
{
    orc_prob *P = (orc_prob *)h;
    int nx = P->n[0], ny = P->n[1], nz = P->n[2];
    for (i64 e = 0; e < P->nn; ++e) y[e] = 0.0;
    for (int k = 1; k < nz - 1; ++k)
        for (int j = 1; j < ny - 1; ++j)
            for (int i = 1; i < nx - 1; ++i) {
                i64 e = nid(P, i, j, k);
                if (P->type[e] == T_REG) {
                    double A[27], q[27];
                    int off[27][3];
                    regular_row(P, i, j, k, A, q, off);
                    double s = 0.0;
                    for (int m = 0; m < 27; ++m) {
                        i64 nb = nid(P, i + off[m][0], j + off[m][1], k + off[m][2]);
                        if (is_unknown(P, nb)) s += A[m] * x[nb];
                    }
                    y[e] = s;
                } else if (P->type[e] == T_IRR) {
                    i64 r = P->irr_of_node[e];
                    double s = 0.0;
                    for (i64 q = P->irr_ptr[r]; q < P->irr_ptr[r + 1]; ++q) s += P->irr_val[q] * x[P->irr_col[q]];
                    y[e] = s;
                }
            }
}

/* K row coefficients at node e, using the stored Shortley-Weller rows at irregular nodes */
static void k_coef(const orc_prob *P, i64 e, const int c[3], double coef[7])
{
    if (P->type[e] == T_IRR) {
        memcpy(coef, &P->ksw[7 * P->irr_of_node[e]], sizeof(double) * 7);
        return;
    }
    coef[0] = 0.0;
    for (int d = 0; d < 3; ++d) {
        coef[0] += P->Kb[d][c[d]];
        i64 nm = e - P->stride[d], np_ = e + P->stride[d];
        coef[1 + 2 * d] = is_unknown(P, nm) ? P->Ka[d][c[d]] : 0.0;
        coef[2 + 2 * d] = is_unknown(P, np_) ? P->Kc[d][c[d]] : 0.0;
    }
}

/* y = K x on unknown nodes */
void orc_apply_K(void *h, const double *x, double *y)
{
    orc_prob *P = (orc_prob *)h;
    for (i64 e = 0; e < P->nn; ++e) {
        y[e] = 0.0;
        if (!is_unknown(P, e)) continue;
        int c[3];
        coords_of(P, e, c);
        double co[7];
        k_coef(P, e, c, co);
        double s = co[0] * x[e];
        for (int d = 0; d < 3; ++d) {
            s += co[1 + 2 * d] * x[e - P->stride[d]];
            s += co[2 + 2 * d] * x[e + P->stride[d]];
        }
        y[e] = s;
    }
}

/* Chebyshev coefficients: x_{k+1} = x_k + c1[k] (x_k - x_{k-1}) + c2[k] D^{-1}(b - A x_k),
 * for the spectrum of D^{-1}A in [lo, hi] (Saad, Alg. 12.1); c1[0] = 0, c2[0] = 1/theta. */
static void cheb_coef(int iters, double lo, double hi, double *c1, double *c2)
{
    double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho_prev = 1.0 / sigma;
    c1[0] = 0.0;
    c2[0] = 1.0 / theta;
    for (int k = 1; k < iters; ++k) {
        double rho = 1.0 / (2.0 * sigma - rho_prev);
        c1[k] = rho * rho_prev;
        c2[k] = 2.0 * rho / delta;
        rho_prev = rho;
    }
}

/* `iters` Chebyshev-Jacobi steps on K x = rho from the initial guess in x (in place), for the
 * spectrum of diag(K)^{-1} K in [lo, hi]: the multigrid smoother. */
void orc_smooth(void *h, const double *rho, double *x, int iters, double lo, double hi)
{
    orc_prob *P = (orc_prob *)h;
    double c1[64], c2[64];
    if (iters > 64) iters = 64;
    cheb_coef(iters, lo, hi, c1, c2);
    double *xp = dalloc(P->nn), *xc = dalloc(P->nn), *xn = dalloc(P->nn);
    memcpy(xc, x, sizeof(double) * P->nn);
    memcpy(xp, x, sizeof(double) * P->nn);
    for (int it = 0; it < iters; ++it) {
        for (i64 e = 0; e < P->nn; ++e) {
            if (!is_unknown(P, e)) { xn[e] = 0.0; continue; }
            int c[3];
            coords_of(P, e, c);
            double co[7];
            k_coef(P, e, c, co);
            double kx = co[0] * xc[e];
            for (int d = 0; d < 3; ++d) kx += co[1 + 2 * d] * xc[e - P->stride[d]] + co[2 + 2 * d] * xc[e + P->stride[d]];
            xn[e] = xc[e] + c1[it] * (xc[e] - xp[e]) + c2[it] * (rho[e] - kx) / co[0];
        }
        double *tmp = xp; xp = xc; xc = xn; xn = tmp;
    }
    memcpy(x, xc, sizeof(double) * P->nn);
    free(xp); free(xc); free(xn);
}

/* phi ~= K^{-1} rho: `iters` Chebyshev-Jacobi steps from phi_0 = 0 on -K phi = -rho
 * (D = -diag K > 0), with spectrum bounds [lo, hi] of D^{-1}(-K). */
void orc_precond(void *h, const double *rho, double *phi, int iters, double lo, double hi)
{
    orc_prob *P = (orc_prob *)h;
    double c1[64], c2[64];
    if (iters > 64) iters = 64;
    cheb_coef(iters, lo, hi, c1, c2);
    double *xp = dalloc(P->nn), *xc = dalloc(P->nn), *xn = dalloc(P->nn);
    for (int it = 0; it < iters; ++it) {
        for (i64 e = 0; e < P->nn; ++e) {
            if (!is_unknown(P, e)) { xn[e] = 0.0; continue; }
            int c[3];
            coords_of(P, e, c);
            double co[7];
            k_coef(P, e, c, co);
            double kx = co[0] * xc[e];
            for (int d = 0; d < 3; ++d) kx += co[1 + 2 * d] * xc[e - P->stride[d]] + co[2 + 2 * d] * xc[e + P->stride[d]];
            /* D^{-1}(b - A x) with A = -K, b = -rho, D = -diag K */
            double z = (rho[e] - kx) / co[0];
            xn[e] = xc[e] + c1[it] * (xc[e] - xp[e]) + c2[it] * z;
        }
        double *tmp = xp; xp = xc; xc = xn; xn = tmp;
    }
    memcpy(phi, xc, sizeof(double) * P->nn);
    free(xp); free(xc); free(xn);
}

/* ------------------------------------------------------------------------------------ */
/* Strongly implicit procedure for K phi = rho (the family of the paper's inner solver)  */
/* ------------------------------------------------------------------------------------ */
/* Sec. 3.3 solves the preconditioned system with the modified strongly implicit procedure
 * of Zedan & Schneider (ref. 24), whose recurrences the paper does not give.  This is the
 * strongly implicit procedure in its original form (Stone's partial-cancellation incomplete
 * factorisation, extended to the 7-point operator in three dimensions), derived here:
 *
 * K is approximated by M = L U with L lower triangular (entries b, c, d at the -z, -y, -x
 * neighbours B, S, W and e on the diagonal) and U upper triangular with unit diagonal
 * (entries f, g, h at the +x, +y, +z neighbours E, N, T), unknowns in lexicographic order
 * (x fastest).  L U has, besides K's seven positions, six more at B+E, B+N, S+E, S+T, W+N,
 * W+T with values X1 = b f_B, X2 = b g_B, X3 = c f_S, X4 = c h_S, X5 = d g_W, X6 = d h_W.
 * The value of the unknown at such a position is approximated by the first-order Taylor
 * combination of two stencil points, phi_{Q+R} ~ alpha (phi_Q + phi_R - phi_P), and M is
 * made to equal K at K's positions with those terms moved onto them:
 *   b = K_B / (1 + alpha (f_B + g_B)),  c = K_S / (1 + alpha (f_S + h_S)),
 *   d = K_W / (1 + alpha (g_W + h_W)),
 *   e = K_P - b h_B - c g_S - d f_W + alpha (X1 + ... + X6),
 *   f = (K_E - alpha (X1 + X3)) / e,  g = (K_N - alpha (X2 + X5)) / e,
 *   h = (K_T - alpha (X4 + X6)) / e,
 * with every factor entry toward a node that is not an unknown (wall or solid) taken as 0.
 * alpha = 0 gives the incomplete factorisation with no fill, ILU(0).  One iteration: r =
 * rho - K phi, L v = r (forward, increasing order), U delta = v (backward), phi += delta;
 * from phi = 0, a fixed number of iterations is a fixed linear map of rho. */

/* factors per node: out[7 e + q], q = b, c, d, e, f, g, h (0 at nodes that are not unknowns) */
void orc_sip_factor(void *h, double alpha, double *out)
{
    orc_prob *P = (orc_prob *)h;
    memset(out, 0, sizeof(double) * 7 * (size_t)P->nn);
    for (i64 e = 0; e < P->nn; ++e) {
        if (!is_unknown(P, e)) continue;
        int c[3];
        coords_of(P, e, c);
        double co[7];
        k_coef(P, e, c, co);
        const i64 nB = e - P->stride[2], nS = e - P->stride[1], nW = e - 1;
        const double *FB = out + 7 * nB, *FS = out + 7 * nS, *FW = out + 7 * nW;
        /* factor entries of neighbours that are not unknowns are 0 (out is zeroed there) */
        double b = co[5] / (1.0 + alpha * (FB[4] + FB[5]));
        double cc = co[3] / (1.0 + alpha * (FS[4] + FS[6]));
        double d = co[1] / (1.0 + alpha * (FW[5] + FW[6]));
        double X1 = b * FB[4], X2 = b * FB[5], X3 = cc * FS[4], X4 = cc * FS[6], X5 = d * FW[5], X6 = d * FW[6];
        double ee = co[0] - b * FB[6] - cc * FS[5] - d * FW[4] + alpha * (X1 + X2 + X3 + X4 + X5 + X6);
        double *F = out + 7 * e;
        F[0] = b;
        F[1] = cc;
        F[2] = d;
        F[3] = ee;
        F[4] = is_unknown(P, e + 1) ? (co[2] - alpha * (X1 + X3)) / ee : 0.0;
        F[5] = is_unknown(P, e + P->stride[1]) ? (co[4] - alpha * (X2 + X5)) / ee : 0.0;
        F[6] = is_unknown(P, e + P->stride[2]) ? (co[6] - alpha * (X4 + X6)) / ee : 0.0;
    }
}

/* phi = `iters` iterations of the strongly implicit procedure from phi = 0 with the
 * factors of orc_sip_factor */
void orc_sip_precond(void *h, const double *F, const double *rho, double *phi, int iters)
{
    orc_prob *P = (orc_prob *)h;
    i64 nn = P->nn;
    double *r = dalloc(nn), *v = dalloc(nn);
    memset(phi, 0, sizeof(double) * nn);
    for (int it = 0; it < iters; ++it) {
        orc_apply_K(P, phi, r);
        for (i64 e = 0; e < nn; ++e) r[e] = is_unknown(P, e) ? rho[e] - r[e] : 0.0;
        for (i64 e = 0; e < nn; ++e) {             /* L v = r */
            if (!is_unknown(P, e)) { v[e] = 0.0; continue; }
            const double *Fe = F + 7 * e;
            v[e] = (r[e] - Fe[0] * v[e - P->stride[2]] - Fe[1] * v[e - P->stride[1]] - Fe[2] * v[e - 1]) / Fe[3];
        }
        for (i64 e = nn - 1; e >= 0; --e) {        /* U delta = v (delta in v) */
            if (!is_unknown(P, e)) continue;
            const double *Fe = F + 7 * e;
            v[e] -= Fe[4] * v[e + 1] + Fe[5] * v[e + P->stride[1]] + Fe[6] * v[e + P->stride[2]];
        }
        for (i64 e = 0; e < nn; ++e)
            if (is_unknown(P, e)) phi[e] += v[e];
    }
    free(r);
    free(v);
}

/* ------------------------------------------------------------------------------------ */
/* BiCGSTAB (Alg. 1 with the split of Eq. Bdec)                                          */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int inner_iters;      /* preconditioner steps per apply */
    int max_iters;        /* cap on BiCGSTAB iterations (all refinement steps together) */
    int mixed;            /* 0: plain FP64; 1: FP64 refinement around an inner solve with FP32 storage */
    int max_refine;
    int max_restarts;
    double lam_lo, lam_hi;
    double inner_tol;     /* per refinement step relative reduction */
} orc_opts;

/* out stats: [iters, refine_steps, restarts, rel_residual] */

static double dot(const orc_prob *P, const double *a, const double *b)
{
    double s = 0.0;
    for (i64 e = 0; e < P->nn; ++e)
        if (is_unknown(P, e)) s += a[e] * b[e];
    return s;
}

/* diagonal entry of B at an unknown node (the (0,0,0) coefficient of its row) */
static double b_diag(const orc_prob *P, i64 e)
{
    if (P->type[e] == T_IRR) {
        i64 r = P->irr_of_node[e];
        for (i64 q = P->irr_ptr[r]; q < P->irr_ptr[r + 1]; ++q)
            if (P->irr_col[q] == e) return P->irr_val[q];
        return 1.0;
    }
    int c[3];
    coords_of(P, e, c);
    return P->Rb[0][c[0]] + P->Rb[1][c[1]] + P->Rb[2][c[2]];
}

/* ||D^{-1} a||_2 over unknowns, D = diag(B): the Jacobi-weighted norm of the stop test */
static double snorm(const orc_prob *P, const double *a)
{
    double s = 0.0;
    for (i64 e = 0; e < P->nn; ++e)
        if (is_unknown(P, e)) {
            double v = a[e] / b_diag(P, e);
            s += v * v;
        }
    return sqrt(s);
}

/* true residual t = rhs - B x; returns ||t||_2, *sn = ||D^{-1} t||_2 */
static double true_res(orc_prob *P, const double *rhs, const double *x, double *t, double *sn)
{
    orc_apply(P, x, t);
    double s2 = 0.0;
    for (i64 e = 0; e < P->nn; ++e) {
        t[e] = is_unknown(P, e) ? rhs[e] - t[e] : 0.0;
        s2 += t[e] * t[e];
    }
    *sn = snorm(P, t);
    return sqrt(s2);
}

/* round to FP32 storage when fp32 is set */
static void store(double *v, i64 nn, int fp32)
{
    if (!fp32) return;
    for (i64 e = 0; e < nn; ++e) v[e] = (double)(float)v[e];
}

/* One BiCGSTAB solve of B x = rhs from x (in/out).  The recursion is Alg. 1 on the
 * paper-scaled B; it stops when the Jacobi-weighted residual ||D^{-1} r|| <= stop_s, and the
 * true residual must then satisfy both ||D^{-1} r|| <= stop_s and ||r|| <= stop_p.
 * Returns 0 converged, 1 max iterations, 2 breakdown.  *it counts iterations. */
static int bicgstab(orc_prob *P, const double *rhs, double *x, double stop_s, double stop_p, const orc_opts *o,
                    int fp32, int *it, int max_it, int *restarts)
{
    i64 nn = P->nn;
    double *r = dalloc(nn), *r0 = dalloc(nn), *p = dalloc(nn), *ph = dalloc(nn), *v = dalloc(nn);
    double *s = dalloc(nn), *sh = dalloc(nn), *t = dalloc(nn);
    int status = 1;
    for (int rs = 0;; ++rs) {
        double sn, pn = true_res(P, rhs, x, r, &sn);
        store(r, nn, fp32);
        if (sn <= stop_s && pn <= stop_p) { status = 0; break; }
        if (rs > o->max_restarts) { status = 1; break; }
        if (rs > 0) (*restarts)++;
        memcpy(r0, r, sizeof(double) * nn);
        memcpy(p, r, sizeof(double) * nn);
        double rho = dot(P, r0, r);
        int broke = 0;
        while (*it < max_it) {
            orc_precond(P, p, ph, o->inner_iters, o->lam_lo, o->lam_hi);
            store(ph, nn, fp32);
            orc_apply(P, ph, v);
            store(v, nn, fp32);
            double sig = dot(P, r0, v);
            if (sig == 0.0 || fabs(sig) <= 1e-30 * sqrt(dot(P, r0, r0) * dot(P, v, v))) { broke = 1; break; }
            double alpha = rho / sig;
            for (i64 e = 0; e < nn; ++e) s[e] = r[e] - alpha * v[e];
            store(s, nn, fp32);
            orc_precond(P, s, sh, o->inner_iters, o->lam_lo, o->lam_hi);
            store(sh, nn, fp32);
            orc_apply(P, sh, t);
            store(t, nn, fp32);
            double tt = dot(P, t, t), ts = dot(P, t, s);
            double omega = tt > 0.0 ? ts / tt : 0.0;
            for (i64 e = 0; e < nn; ++e) {
                x[e] += alpha * ph[e] + omega * sh[e];
                r[e] = s[e] - omega * t[e];
            }
            store(x, nn, fp32);
            store(r, nn, fp32);
            (*it)++;
            if (snorm(P, r) <= stop_s) break;
            if (omega == 0.0) { broke = 1; break; }
            double rho_new = dot(P, r0, r);
            double beta = (alpha / omega) * (rho_new / rho);
            rho = rho_new;
            for (i64 e = 0; e < nn; ++e) p[e] = r[e] + beta * (p[e] - omega * v[e]);
            store(p, nn, fp32);
        }
        if (broke) status = 2;
        if (*it >= max_it) {
            double sn2, pn2 = true_res(P, rhs, x, t, &sn2);
            status = (sn2 <= stop_s && pn2 <= stop_p) ? 0 : (broke ? 2 : 1);
            break;
        }
    }
    free(r); free(r0); free(p); free(ph); free(v); free(s); free(sh); free(t);
    return status;
}

/* Solve B u = rhs to ||r||/||b|| <= tol and ||D^{-1} r||/||D^{-1} b|| <= tol.
 * u: all nodes; in = warm start at unknown nodes, out = solution at unknowns, g at wall
 * nodes, 0 at solid nodes.  stats: [iters, refine_steps, restarts, rel_res, rel_res_jacobi].
 * Returns 0 converged, -5 breakdown, -6 not converged. */
int orc_solve(void *h, double tol, double *u, const orc_opts *o, double *stats)
{
    orc_prob *P = (orc_prob *)h;
    i64 nn = P->nn;
    double *x = dalloc(nn), *t = dalloc(nn);
    for (i64 e = 0; e < nn; ++e) x[e] = is_unknown(P, e) ? u[e] : 0.0;
    double bn = sqrt(dot(P, P->rhs, P->rhs)), bs = snorm(P, P->rhs);
    if (bn == 0.0) bn = 1.0;
    if (bs == 0.0) bs = 1.0;
    int it = 0, restarts = 0, refine = 0, status;
    if (!o->mixed) {
        status = bicgstab(P, P->rhs, x, tol * bs, tol * bn, o, 0, &it, o->max_iters, &restarts);
    } else {
        double *r = dalloc(nn), *d = dalloc(nn);
        status = 1;
        for (refine = 0; refine < o->max_refine; ++refine) {
            double sn, pn = true_res(P, P->rhs, x, r, &sn);
            if (sn <= tol * bs && pn <= tol * bn) { status = 0; break; }
            if (it >= o->max_iters) break;
            store(r, nn, 1);
            memset(d, 0, sizeof(double) * nn);
            double target = o->inner_tol * sn;
            if (target < 0.5 * tol * bs) target = 0.5 * tol * bs;
            int st = bicgstab(P, r, d, target, HUGE_VAL, o, 1, &it, o->max_iters, &restarts);
            for (i64 e = 0; e < nn; ++e) x[e] += d[e];
            if (st == 2) { status = 2; break; }
        }
        if (status == 1) {
            double sn, pn = true_res(P, P->rhs, x, r, &sn);
            if (sn <= tol * bs && pn <= tol * bn) status = 0;
        }
        free(r); free(d);
    }
    double sn, pn = true_res(P, P->rhs, x, t, &sn);
    free(t);
    for (i64 e = 0; e < nn; ++e) {
        if (P->type[e] == T_BOUND) u[e] = P->g[e];
        else if (P->type[e] == T_SOLID) u[e] = 0.0;
        else u[e] = x[e];
    }
    free(x);
    if (stats) {
        stats[0] = it; stats[1] = refine; stats[2] = restarts; stats[3] = pn / bn; stats[4] = sn / bs;
    }
    if (status == 0) return 0;
    return status == 2 ? -5 : -6;
}

/* r = b - B u at unknown nodes (0 elsewhere); *rel = ||r||_2 / ||b||_2 */
void orc_residual(void *h, const double *u, double *r, double *rel)
{
    orc_prob *P = (orc_prob *)h;
    double *t = dalloc(P->nn);
    orc_apply(P, u, t);
    double s2 = 0.0, b2 = 0.0;
    for (i64 e = 0; e < P->nn; ++e) {
        double d = is_unknown(P, e) ? P->rhs[e] - t[e] : 0.0;
        if (r) r[e] = d;
        s2 += d * d;
        if (is_unknown(P, e)) b2 += P->rhs[e] * P->rhs[e];
    }
    free(t);
    *rel = sqrt(s2) / (b2 > 0 ? sqrt(b2) : 1.0);
}

int orc_opts_size(void) { return (int)sizeof(orc_opts); }
