/*
 * net_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain-loop reference of the warm-start network (a 4-level 3D convolutional
 * encoder-decoder) and of its training loss gradient, used to check the GPU kernels.
 * Nothing here is loaded by the GPU library.
 *
 * Network (channels c0..c3, input channels 3, output 1; n = coarse points per direction,
 * divisible by 8):
 *   E_l a/b : two 3x3x3 convolutions (zero padding) with bias and ReLU per level l = 0..3,
 *             inputs of level l > 0 are the 2x2x2 averages of level l-1's output;
 *   D_l a/b : for l = 2, 1, 0: nearest-neighbour x2 upsampling of the level below,
 *             concatenated [upsampled, skip_l], then two 3x3x3 convolutions + ReLU;
 *   head    : 1x1x1 convolution c0 -> 1 with bias, no activation.
 * Layout: activations [B][C][z][y][x]; weights of a layer [co][ci][kz][ky][kx] then bias
 * [co], layers in the order E0a E0b E1a E1b E2a E2b E3a E3b D2a D2b D1a D1b D0a D0b head.
 *
 * BF16 emulation (bf16 != 0) rounds, to nearest even, exactly where the GPU stores BF16:
 * the weights of the 3x3x3 layers, the network input, every stored activation (after
 * ReLU, after pooling), and the gradient entering each 3x3x3 layer's backward pass.
 * Accumulation is in double here (FP32 on the GPU).  With bf16 = 0 everything is double.
 *
 * Loss: L = sum_v m_v (p_v - t_v)^2 / sum_v m_v over all batch entries.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double bf16r(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v;   /* inf / nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static void round_all(double *a, long n, int on)
{
    if (!on) return;
    for (long e = 0; e < n; ++e) a[e] = bf16r(a[e]);
}

/* out[b][co][v] = bias[co] + sum_{ci,tap} W[co][ci][tap] in[b][ci][v + tap - 1] */
static void conv3_fwd(int B, int Ci, int Co, int n, const double *in, const double *W, const double *bias, double *out)
{
    long nv = (long)n * n * n;
    for (int b = 0; b < B; ++b)
        for (int co = 0; co < Co; ++co)
            for (int z = 0; z < n; ++z)
                for (int y = 0; y < n; ++y)
                    for (int x = 0; x < n; ++x) {
                        double s = bias[co];
                        for (int ci = 0; ci < Ci; ++ci)
                            for (int dz = -1; dz <= 1; ++dz)
                                for (int dy = -1; dy <= 1; ++dy)
                                    for (int dx = -1; dx <= 1; ++dx) {
                                        int zz = z + dz, yy = y + dy, xx = x + dx;
                                        if (zz < 0 || yy < 0 || xx < 0 || zz >= n || yy >= n || xx >= n) continue;
                                        double w = W[(((long)co * Ci + ci) * 3 + dz + 1) * 9 + (dy + 1) * 3 + dx + 1];
                                        s += w * in[((long)b * Ci + ci) * nv + ((long)zz * n + yy) * n + xx];
                                    }
                        out[((long)b * Co + co) * nv + ((long)z * n + y) * n + x] = s;
                    }
}

/* given dout: din (may be NULL), dW, dbias accumulated */
static void conv3_bwd(int B, int Ci, int Co, int n, const double *in, const double *W, const double *dout, double *din,
                      double *dW, double *dbias)
{
    long nv = (long)n * n * n;
    if (din) memset(din, 0, sizeof(double) * B * Ci * nv);
    for (int b = 0; b < B; ++b)
        for (int co = 0; co < Co; ++co)
            for (int z = 0; z < n; ++z)
                for (int y = 0; y < n; ++y)
                    for (int x = 0; x < n; ++x) {
                        double g = dout[((long)b * Co + co) * nv + ((long)z * n + y) * n + x];
                        if (g == 0.0) continue;
                        dbias[co] += g;
                        for (int ci = 0; ci < Ci; ++ci)
                            for (int dz = -1; dz <= 1; ++dz)
                                for (int dy = -1; dy <= 1; ++dy)
                                    for (int dx = -1; dx <= 1; ++dx) {
                                        int zz = z + dz, yy = y + dy, xx = x + dx;
                                        if (zz < 0 || yy < 0 || xx < 0 || zz >= n || yy >= n || xx >= n) continue;
                                        long wi = (((long)co * Ci + ci) * 3 + dz + 1) * 9 + (dy + 1) * 3 + dx + 1;
                                        long ii = ((long)b * Ci + ci) * nv + ((long)zz * n + yy) * n + xx;
                                        dW[wi] += g * in[ii];
                                        if (din) din[ii] += g * W[wi];
                                    }
                    }
}

static void pool_fwd(int B, int C, int n, const double *in, double *out)
{
    int m = n / 2;
    for (int b = 0; b < B; ++b)
        for (int c = 0; c < C; ++c)
            for (int z = 0; z < m; ++z)
                for (int y = 0; y < m; ++y)
                    for (int x = 0; x < m; ++x) {
                        double s = 0.0;
                        for (int q = 0; q < 8; ++q)
                            s += in[(((long)b * C + c) * n + 2 * z + (q >> 2)) * n * n + (2 * y + ((q >> 1) & 1)) * n +
                                    2 * x + (q & 1)];
                        out[(((long)b * C + c) * m + z) * m * m + y * m + x] = s / 8.0;
                    }
}

static void pool_bwd(int B, int C, int n, const double *dout, double *din)
{
    int m = n / 2;
    for (int b = 0; b < B; ++b)
        for (int c = 0; c < C; ++c)
            for (int z = 0; z < n; ++z)
                for (int y = 0; y < n; ++y)
                    for (int x = 0; x < n; ++x)
                        din[(((long)b * C + c) * n + z) * n * n + y * n + x] +=
                            dout[(((long)b * C + c) * m + z / 2) * m * m + (y / 2) * m + x / 2] / 8.0;
}

/* out: [B][C0+C1][2m]^3 = [up(lo) (C0 channels), skip (C1 channels)] */
static void up_cat_fwd(int B, int C0, int C1, int m, const double *lo, const double *skip, double *out)
{
    int n = 2 * m;
    long nv = (long)n * n * n;
    for (int b = 0; b < B; ++b) {
        for (int c = 0; c < C0; ++c)
            for (int z = 0; z < n; ++z)
                for (int y = 0; y < n; ++y)
                    for (int x = 0; x < n; ++x)
                        out[((long)b * (C0 + C1) + c) * nv + ((long)z * n + y) * n + x] =
                            lo[(((long)b * C0 + c) * m + z / 2) * m * m + (y / 2) * m + x / 2];
        for (int c = 0; c < C1; ++c)
            memcpy(&out[((long)b * (C0 + C1) + C0 + c) * nv], &skip[((long)b * C1 + c) * nv], sizeof(double) * nv);
    }
}

static void up_cat_bwd(int B, int C0, int C1, int m, const double *dout, double *dlo, double *dskip)
{
    int n = 2 * m;
    long nv = (long)n * n * n;
    for (int b = 0; b < B; ++b) {
        for (int c = 0; c < C0; ++c)
            for (int z = 0; z < n; ++z)
                for (int y = 0; y < n; ++y)
                    for (int x = 0; x < n; ++x)
                        dlo[(((long)b * C0 + c) * m + z / 2) * m * m + (y / 2) * m + x / 2] +=
                            dout[((long)b * (C0 + C1) + c) * nv + ((long)z * n + y) * n + x];
        for (int c = 0; c < C1; ++c)
            for (long v = 0; v < nv; ++v)
                dskip[((long)b * C1 + c) * nv + v] += dout[((long)b * (C0 + C1) + C0 + c) * nv + v];
    }
}

#define NCONV 14

/* per-layer (ci, co, level) of the 3x3x3 layers */
static void layer_dims(const int ch[4], int cin, int L, int *ci, int *co, int *lvl)
{
    static const int lv[NCONV] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0};
    *lvl = lv[L];
    switch (L) {
    case 0: *ci = cin; *co = ch[0]; break;
    case 1: *ci = ch[0]; *co = ch[0]; break;
    case 2: *ci = ch[0]; *co = ch[1]; break;
    case 3: *ci = ch[1]; *co = ch[1]; break;
    case 4: *ci = ch[1]; *co = ch[2]; break;
    case 5: *ci = ch[2]; *co = ch[2]; break;
    case 6: *ci = ch[2]; *co = ch[3]; break;
    case 7: *ci = ch[3]; *co = ch[3]; break;
    case 8: *ci = ch[3] + ch[2]; *co = ch[2]; break;
    case 9: *ci = ch[2]; *co = ch[2]; break;
    case 10: *ci = ch[2] + ch[1]; *co = ch[1]; break;
    case 11: *ci = ch[1]; *co = ch[1]; break;
    case 12: *ci = ch[1] + ch[0]; *co = ch[0]; break;
    default: *ci = ch[0]; *co = ch[0]; break;
    }
}

long onet_param_count(const int ch[4], int cin)
{
    long n = 0;
    for (int L = 0; L < NCONV; ++L) {
        int ci, co, lv;
        layer_dims(ch, cin, L, &ci, &co, &lv);
        n += (long)co * ci * 27 + co;
    }
    return n + ch[0] + 1;
}

/* Forward, loss and (if grad != NULL) the gradient of the loss w.r.t. every parameter.
 * input [B][cin][n^3], target/mask [B][n^3] (mask may be NULL = all ones), pred [B][n^3]
 * (may be NULL).  Returns the loss. */
double onet_run(const int ch[4], int cin, int B, int n, const double *params, const double *input,
                const double *target, const double *mask, int bf16, double *pred, double *grad)
{
    int ci, co, lv;
    long off[NCONV + 1];
    long o = 0;
    for (int L = 0; L < NCONV; ++L) {
        layer_dims(ch, cin, L, &ci, &co, &lv);
        off[L] = o;
        o += (long)co * ci * 27 + co;
    }
    off[NCONV] = o;   /* head: weights ch[0], bias 1 */
    long np = o + ch[0] + 1;
    double *P = (double *)malloc(sizeof(double) * np);
    memcpy(P, params, sizeof(double) * np);
    for (int L = 0; L < NCONV; ++L) {
        layer_dims(ch, cin, L, &ci, &co, &lv);
        round_all(P + off[L], (long)co * ci * 27, bf16);   /* 3x3x3 weights are BF16 on the GPU */
    }
    long nvs[4];
    for (int l = 0; l < 4; ++l) {
        long m = n >> l;
        nvs[l] = m * m * m;
    }
    /* activations: in[L] (input of layer L), out[L] (after ReLU, stored) */
    double *in[NCONV], *out[NCONV];
    for (int L = 0; L < NCONV; ++L) {
        layer_dims(ch, cin, L, &ci, &co, &lv);
        in[L] = (double *)calloc((size_t)B * ci * nvs[lv], sizeof(double));
        out[L] = (double *)calloc((size_t)B * co * nvs[lv], sizeof(double));
    }
    double *x0 = in[0];
    memcpy(x0, input, sizeof(double) * B * cin * nvs[0]);
    round_all(x0, (long)B * cin * nvs[0], bf16);
    for (int L = 0; L < NCONV; ++L) {
        layer_dims(ch, cin, L, &ci, &co, &lv);
        int m = n >> lv;
        if (L > 0) {
            int pci, pco, plv;
            layer_dims(ch, cin, L - 1, &pci, &pco, &plv);
            if (L == 2 || L == 4 || L == 6) {           /* pool the level above */
                pool_fwd(B, pco, m * 2, out[L - 1], in[L]);
                round_all(in[L], (long)B * ci * nvs[lv], bf16);
            } else if (L == 8 || L == 10 || L == 12) {   /* upsample + concat skip */
                int skipL = (L == 8) ? 5 : (L == 10) ? 3 : 1;
                int sci, sco, slv;
                layer_dims(ch, cin, skipL, &sci, &sco, &slv);
                up_cat_fwd(B, pco, sco, m / 2, out[L - 1], out[skipL], in[L]);
            } else {
                memcpy(in[L], out[L - 1], sizeof(double) * B * ci * nvs[lv]);
            }
        }
        conv3_fwd(B, ci, co, m, in[L], P + off[L], P + off[L] + (long)co * ci * 27, out[L]);
        for (long e = 0; e < (long)B * co * nvs[lv]; ++e) out[L][e] = out[L][e] > 0.0 ? out[L][e] : 0.0;
        round_all(out[L], (long)B * co * nvs[lv], bf16);
    }
    /* head */
    double *p = (double *)calloc((size_t)B * nvs[0], sizeof(double));
    const double *hw = P + off[NCONV];
    for (int b = 0; b < B; ++b)
        for (long v = 0; v < nvs[0]; ++v) {
            double s = hw[ch[0]];
            for (int c = 0; c < ch[0]; ++c) s += hw[c] * out[NCONV - 1][((long)b * ch[0] + c) * nvs[0] + v];
            p[(long)b * nvs[0] + v] = s;
        }
    if (pred) memcpy(pred, p, sizeof(double) * B * nvs[0]);
    double msum = 0.0, loss = 0.0;
    for (long e = 0; e < (long)B * nvs[0]; ++e) {
        double m = mask ? mask[e] : 1.0;
        msum += m;
        loss += m * (p[e] - target[e]) * (p[e] - target[e]);
    }
    loss /= msum;
    if (grad) {
        memset(grad, 0, sizeof(double) * np);
        double *dp = (double *)calloc((size_t)B * nvs[0], sizeof(double));
        for (long e = 0; e < (long)B * nvs[0]; ++e) dp[e] = 2.0 * (mask ? mask[e] : 1.0) * (p[e] - target[e]) / msum;
        /* gradients w.r.t. layer outputs (stored activations) */
        double *dout[NCONV];
        for (int L = 0; L < NCONV; ++L) {
            layer_dims(ch, cin, L, &ci, &co, &lv);
            dout[L] = (double *)calloc((size_t)B * co * nvs[lv], sizeof(double));
        }
        double *gh = grad + off[NCONV];
        for (int b = 0; b < B; ++b)
            for (long v = 0; v < nvs[0]; ++v) {
                double g = dp[(long)b * nvs[0] + v];
                gh[ch[0]] += g;
                for (int c = 0; c < ch[0]; ++c) {
                    gh[c] += g * out[NCONV - 1][((long)b * ch[0] + c) * nvs[0] + v];
                    dout[NCONV - 1][((long)b * ch[0] + c) * nvs[0] + v] += g * hw[c];
                }
            }
        for (int L = NCONV - 1; L >= 0; --L) {
            layer_dims(ch, cin, L, &ci, &co, &lv);
            int m = n >> lv;
            long nout = (long)B * co * nvs[lv];
            double *g = (double *)malloc(sizeof(double) * nout);
            for (long e = 0; e < nout; ++e) g[e] = out[L][e] > 0.0 ? dout[L][e] : 0.0;   /* ReLU */
            round_all(g, nout, bf16);
            double *din = (double *)calloc((size_t)B * ci * nvs[lv], sizeof(double));
            conv3_bwd(B, ci, co, m, in[L], P + off[L], g, L > 0 ? din : NULL, grad + off[L],
                      grad + off[L] + (long)co * ci * 27);
            free(g);
            if (L > 0) {
                int pci, pco, plv;
                layer_dims(ch, cin, L - 1, &pci, &pco, &plv);
                if (L == 2 || L == 4 || L == 6) {
                    pool_bwd(B, pco, m * 2, din, dout[L - 1]);
                } else if (L == 8 || L == 10 || L == 12) {
                    int skipL = (L == 8) ? 5 : (L == 10) ? 3 : 1;
                    int sci, sco, slv;
                    layer_dims(ch, cin, skipL, &sci, &sco, &slv);
                    up_cat_bwd(B, pco, sco, m / 2, din, dout[L - 1], dout[skipL]);
                } else {
                    for (long e = 0; e < (long)B * ci * nvs[lv]; ++e) dout[L - 1][e] += din[e];
                }
            }
            free(din);
        }
        for (int L = 0; L < NCONV; ++L) free(dout[L]);
        free(dp);
    }
    for (int L = 0; L < NCONV; ++L) {
        free(in[L]);
        free(out[L]);
    }
    free(p);
    free(P);
    return loss;
}

/* single-layer references for unit tests */
void onet_conv3(int B, int Ci, int Co, int n, const double *in, const double *W, const double *bias, double *out)
{
    conv3_fwd(B, Ci, Co, n, in, W, bias, out);
}

void onet_conv3_bwd(int B, int Ci, int Co, int n, const double *in, const double *W, const double *dout, double *din,
                    double *dW, double *dbias)
{
    memset(dW, 0, sizeof(double) * Co * Ci * 27);
    memset(dbias, 0, sizeof(double) * Co);
    conv3_bwd(B, Ci, Co, n, in, W, dout, din, dW, dbias);
}

double onet_bf16(double v) { return bf16r(v); }
