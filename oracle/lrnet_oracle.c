/*
 * CPU oracle for the learned stand-in of the left-right check.
 *
 * TEST INFRASTRUCTURE ONLY (see sgm_oracle.c): loaded by the test suite, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product path.
 *
 * The paper has no learned component; the left-right check it describes
 * (Sec. 3.1) is what this network imitates, and its labels come from that
 * check.  Definitions, stated once and used by both sides:
 *
 * Features per pixel (x, y), FP32, layout feat[(y * W + x) * 4 + k]:
 *   k=0: I_L(x, y) / 255
 *   k=1: d* / (D - 1)                       (d* = WTA disparity)
 *   k=2: S_min / (8 * (62 + P2))            (S_min = S(p, d*))
 *   k=3: S_2 / max(S_min, 1)                (S_2 = min of S(p, d) over
 *                                            |d - d*| >= 2; S_min if none)
 *   each an FP32 division of two exactly representable values.
 *
 * Network: four 3x3 cross-correlation layers with zero padding ("same"),
 * channels 4 -> 16 -> 16 -> 16 -> 1, ReLU after layers 1-3, logit output;
 * probability of "LR-valid" = sigmoid(logit).  Parameters (flat FP32 master
 * vector, 5377 values): W1[16][4][3][3], b1[16], W2[16][16][3][3], b2[16],
 * W3[16][16][3][3], b3[16], W4[1][16][3][3], b4[1].
 *
 * Precision: the layer inputs a0 (features) and a1..a3 (ReLU outputs) and the
 * weights are rounded to BF16 (round to nearest, ties to even); biases stay
 * FP32; each pre-activation is an exact-product sum formed here in FP64 and
 * then rounded to FP32 (the GPU forms it in FP32).
 *
 * Loss: mean over all pixels of BCE-with-logits, softplus(z) - y z.
 * Backward: dL/dz4 = (sigmoid(z4) - y) / N in FP32; the rounding to BF16 is
 * passed straight through; the gradients w.r.t. the pre-activations of layers
 * 3, 2, 1 are rounded to BF16 (they feed BF16 matrix products on the GPU);
 * weight and bias gradients are sums of exact products formed in FP64 here
 * and rounded once to FP32.
 *
 * With round_bf16 = 0 every rounding above is skipped; finite differences of
 * the loss then pin the backward formulas.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NP_W1 (16 * 4 * 9)
#define NP_W2 (16 * 16 * 9)
#define NP_W4 (16 * 9)
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NP_W1)
#define OFF_W2 (OFF_B1 + 16)
#define OFF_B2 (OFF_W2 + NP_W2)
#define OFF_W3 (OFF_B2 + 16)
#define OFF_B3 (OFF_W3 + NP_W2)
#define OFF_W4 (OFF_B3 + 16)
#define OFF_B4 (OFF_W4 + NP_W4)
#define NPARAM (OFF_B4 + 1)

int oracle_lrnet_nparams(void) { return NPARAM; }

/* BF16 round-to-nearest-even from the format definition: keep the upper 16
 * bits of the IEEE binary32 pattern, rounding on the lower 16. */
float oracle_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {
        if (u & 0x007fffffu) u |= 0x00400000u; /* NaN stays NaN */
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u = (u + 0x7fffu + lsb) & 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, 4);
    return r;
}

static float maybe_bf16(float x, int on) { return on ? oracle_bf16(x) : x; }

void oracle_features(const uint8_t *img, int pitch, const uint16_t *S, const int16_t *wta, int H,
                     int W, int D, int P2, float *feat)
{
    float smax_norm = (float)(8 * (62 + P2));
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            const uint16_t *s = S + i * D;
            int ds = wta[i];
            int smin = s[ds];
            int s2 = -1;
            for (int d = 0; d < D; ++d) {
                int gap = d - ds;
                if (gap < 0) gap = -gap;
                if (gap >= 2 && (s2 < 0 || s[d] < s2)) s2 = s[d];
            }
            if (s2 < 0) s2 = smin;
            feat[i * 4 + 0] = (float)img[(size_t)y * pitch + x] / 255.0f;
            feat[i * 4 + 1] = D > 1 ? (float)ds / (float)(D - 1) : 0.0f;
            feat[i * 4 + 2] = (float)smin / smax_norm;
            feat[i * 4 + 3] = (float)s2 / (float)(smin > 1 ? smin : 1);
        }
}

/* z[co][y][x] = b[co] + sum_{ci,ky,kx} w[co][ci][ky][kx] * a[ci][y+ky-1][x+kx-1]
 * (activations channel-major inside the oracle: a[(c * H + y) * W + x]). */
static void conv_fwd(const float *a, int Cin, int H, int W, const float *w, const float *b,
                     int Cout, float *z)
{
    for (int co = 0; co < Cout; ++co)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int ci = 0; ci < Cin; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int yy = y + ky - 1, xx = x + kx - 1;
                            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                            acc += (double)w[((co * Cin + ci) * 3 + ky) * 3 + kx] *
                                   (double)a[((size_t)ci * H + yy) * W + xx];
                        }
                z[((size_t)co * H + y) * W + x] = (float)(acc + (double)b[co]);
            }
}

/* Gradient of the loss w.r.t. the layer input: ga[ci][q] = sum over co and
 * taps k of w[co][ci][k] * gz[co][q - k + 1]. */
static void conv_bwd_data(const float *gz, int Cout, int H, int W, const float *w, int Cin,
                          double *ga)
{
    for (int ci = 0; ci < Cin; ++ci)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int co = 0; co < Cout; ++co)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int yy = y - ky + 1, xx = x - kx + 1;
                            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                            acc += (double)w[((co * Cin + ci) * 3 + ky) * 3 + kx] *
                                   (double)gz[((size_t)co * H + yy) * W + xx];
                        }
                ga[((size_t)ci * H + y) * W + x] = acc;
            }
}

/* dW[co][ci][ky][kx] += sum_p gz[co][p] * a[ci][p + k - 1]; db[co] += sum_p gz[co][p]. */
static void conv_bwd_weight(const float *gz, int Cout, int H, int W, const float *a, int Cin,
                            double *dw, double *db)
{
    for (int co = 0; co < Cout; ++co) {
        for (int ci = 0; ci < Cin; ++ci)
            for (int ky = 0; ky < 3; ++ky)
                for (int kx = 0; kx < 3; ++kx) {
                    double acc = 0.0;
                    for (int y = 0; y < H; ++y)
                        for (int x = 0; x < W; ++x) {
                            int yy = y + ky - 1, xx = x + kx - 1;
                            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                            acc += (double)gz[((size_t)co * H + y) * W + x] *
                                   (double)a[((size_t)ci * H + yy) * W + xx];
                        }
                    dw[((co * Cin + ci) * 3 + ky) * 3 + kx] += acc;
                }
        double s = 0.0;
        for (size_t p = 0; p < (size_t)H * W; ++p) s += (double)gz[(size_t)co * H * W + p];
        db[co] += s;
    }
}

/*
 * Forward (and, if grad != NULL, backward) over a batch of B images.
 * feat [B][H][W][4] FP32, label [B][H][W] in {0, 1} (may be NULL when grad is
 * NULL), params [5377] FP32 master weights.  logits [B][H][W] (optional).
 * Returns the mean loss (or 0 when label is NULL).  grad [5377] FP32.
 */
static double lrnet_run(const float *feat, const uint8_t *label, const float *dz4, int B, int H,
                        int W, const float *params, int round_bf16, float *grad, float *logits);

double oracle_lrnet(const float *feat, const uint8_t *label, int B, int H, int W,
                    const float *params, int round_bf16, float *grad, float *logits)
{
    return lrnet_run(feat, label, NULL, B, H, W, params, round_bf16, grad, logits);
}

/* Backward from a given dL/dz4 [B][H][W] (FP32) instead of the loss: the same
 * forward, then the same backward steps as oracle_lrnet with g4 := dz4. */
void oracle_lrnet_backward(const float *feat, const float *dz4, int B, int H, int W,
                           const float *params, int round_bf16, float *grad)
{
    lrnet_run(feat, NULL, dz4, B, H, W, params, round_bf16, grad, NULL);
}

static double lrnet_run(const float *feat, const uint8_t *label, const float *dz4, int B, int H,
                        int W, const float *params, int round_bf16, float *grad, float *logits)
{
    size_t hw = (size_t)H * W;
    float wq[NPARAM];
    for (int i = 0; i < NPARAM; ++i) wq[i] = params[i];
    /* Weights are used in BF16, biases in FP32. */
    for (int i = 0; i < NP_W1; ++i) wq[OFF_W1 + i] = maybe_bf16(params[OFF_W1 + i], round_bf16);
    for (int i = 0; i < NP_W2; ++i) wq[OFF_W2 + i] = maybe_bf16(params[OFF_W2 + i], round_bf16);
    for (int i = 0; i < NP_W2; ++i) wq[OFF_W3 + i] = maybe_bf16(params[OFF_W3 + i], round_bf16);
    for (int i = 0; i < NP_W4; ++i) wq[OFF_W4 + i] = maybe_bf16(params[OFF_W4 + i], round_bf16);

    float *a0 = malloc(4 * hw * 4), *z1 = malloc(16 * hw * 4), *a1 = malloc(16 * hw * 4);
    float *z2 = malloc(16 * hw * 4), *a2 = malloc(16 * hw * 4), *z3 = malloc(16 * hw * 4);
    float *a3 = malloc(16 * hw * 4), *z4 = malloc(hw * 4);
    float *g4 = malloc(hw * 4), *gz = malloc(16 * hw * 4);
    double *ga = malloc(16 * hw * 8);
    double dparam[NPARAM];
    memset(dparam, 0, sizeof(dparam));
    double loss = 0.0;
    double ntot = (double)B * (double)hw;

    for (int bi = 0; bi < B; ++bi) {
        const float *fb = feat + (size_t)bi * hw * 4;
        for (int c = 0; c < 4; ++c)
            for (size_t p = 0; p < hw; ++p) a0[c * hw + p] = maybe_bf16(fb[p * 4 + c], round_bf16);
        conv_fwd(a0, 4, H, W, wq + OFF_W1, wq + OFF_B1, 16, z1);
        for (size_t i = 0; i < 16 * hw; ++i) a1[i] = maybe_bf16(z1[i] > 0.0f ? z1[i] : 0.0f, round_bf16);
        conv_fwd(a1, 16, H, W, wq + OFF_W2, wq + OFF_B2, 16, z2);
        for (size_t i = 0; i < 16 * hw; ++i) a2[i] = maybe_bf16(z2[i] > 0.0f ? z2[i] : 0.0f, round_bf16);
        conv_fwd(a2, 16, H, W, wq + OFF_W3, wq + OFF_B3, 16, z3);
        for (size_t i = 0; i < 16 * hw; ++i) a3[i] = maybe_bf16(z3[i] > 0.0f ? z3[i] : 0.0f, round_bf16);
        conv_fwd(a3, 16, H, W, wq + OFF_W4, wq + OFF_B4, 1, z4);
        if (logits) memcpy(logits + (size_t)bi * hw, z4, hw * 4);
        if (dz4) {
            memcpy(g4, dz4 + (size_t)bi * hw, hw * 4);
        } else {
            if (!label) continue;
            const uint8_t *lb = label + (size_t)bi * hw;
            for (size_t p = 0; p < hw; ++p) {
                double z = z4[p], y = lb[p] ? 1.0 : 0.0;
                /* softplus(z) - y z, evaluated without overflow */
                double sp = z > 0 ? z + log1p(exp(-z)) : log1p(exp(z));
                loss += sp - y * z;
                double s = 1.0 / (1.0 + exp(-z));
                g4[p] = (float)((s - y) / ntot);
            }
        }
        if (!grad) continue;
        /* layer 4 */
        conv_bwd_weight(g4, 1, H, W, a3, 16, dparam + OFF_W4, dparam + OFF_B4);
        conv_bwd_data(g4, 1, H, W, wq + OFF_W4, 16, ga);
        for (size_t i = 0; i < 16 * hw; ++i)
            gz[i] = maybe_bf16(z3[i] > 0.0f ? (float)ga[i] : 0.0f, round_bf16);
        /* layer 3 */
        conv_bwd_weight(gz, 16, H, W, a2, 16, dparam + OFF_W3, dparam + OFF_B3);
        conv_bwd_data(gz, 16, H, W, wq + OFF_W3, 16, ga);
        for (size_t i = 0; i < 16 * hw; ++i)
            gz[i] = maybe_bf16(z2[i] > 0.0f ? (float)ga[i] : 0.0f, round_bf16);
        /* layer 2 */
        conv_bwd_weight(gz, 16, H, W, a1, 16, dparam + OFF_W2, dparam + OFF_B2);
        conv_bwd_data(gz, 16, H, W, wq + OFF_W2, 16, ga);
        for (size_t i = 0; i < 16 * hw; ++i)
            gz[i] = maybe_bf16(z1[i] > 0.0f ? (float)ga[i] : 0.0f, round_bf16);
        /* layer 1 */
        conv_bwd_weight(gz, 16, H, W, a0, 4, dparam + OFF_W1, dparam + OFF_B1);
    }
    if (grad)
        for (int i = 0; i < NPARAM; ++i) grad[i] = (float)dparam[i];
    free(a0); free(z1); free(a1); free(z2); free(a2); free(z3); free(a3); free(z4);
    free(g4); free(gz); free(ga);
    return label ? loss / ntot : 0.0;
}

/* Adam update in FP32, operations in this order:
 *   m = b1*m + (1-b1)*g;  v = b2*v + (1-b2)*(g*g);
 *   mh = m / (1 - b1t);   vh = v / (1 - b2t);
 *   w = w - (lr * mh) / (sqrtf(vh) + eps)
 * where b1t, b2t are b1, b2 raised to the step count (passed in). */
void oracle_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1,
                 float b2, float eps, float b1t, float b2t)
{
    for (int i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0f - b1) * g[i];
        v[i] = b2 * v[i] + (1.0f - b2) * (g[i] * g[i]);
        float mh = m[i] / (1.0f - b1t);
        float vh = v[i] / (1.0f - b2t);
        w[i] = w[i] - (lr * mh) / (sqrtf(vh) + eps);
    }
}
