/*
 * Drives every entry of the CPU oracle on small seeded inputs, including the
 * degenerate shapes (1x1, one row, one column, D = 1), for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py):
 * any out-of-bounds access, leak or undefined operation aborts the run.
 * Test infrastructure only; the values are not checked here (the pytest pins
 * do that), only that every path runs clean.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_census(const uint8_t *img, int H, int W, int pitch, uint64_t *out);
void oracle_cost(const uint64_t *cb, const uint64_t *cm, int H, int W, int D, int right, uint8_t *cost);
void oracle_path_cost(const uint8_t *cost, int H, int W, int D, int P1, int P2, int dir, int32_t *Lr);
void oracle_aggregate(const uint8_t *cost, int H, int W, int D, int P1, int P2, unsigned mask, uint16_t *S);
void oracle_path_cost_adaptive(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W, int D, int P1,
                               int P2, int dir, int32_t *Lr);
void oracle_aggregate_adaptive(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W, int D, int P1,
                               int P2, unsigned mask, uint16_t *S);
void oracle_wta(const uint16_t *S, int H, int W, int D, int16_t *wta, float *dsub);
void oracle_lr_check(const int16_t *wl, const int16_t *wr, const float *dsub, int H, int W, int tol,
                     uint8_t *valid, float *disp);
void oracle_no_check(const float *dsub, int H, int W, uint8_t *valid, float *disp);
void oracle_wta_right_diag(const uint16_t *S, int H, int W, int D, int16_t *wr);
void oracle_median3x3(const float *in, int H, int W, float *out);
void oracle_combine(const float *d0, const uint8_t *v0, const float *d1, const uint8_t *v1, const float *flow,
                    int H, int W, int has_cam, float f, float B, float cx, float cy, float *sf4, uint8_t *valid,
                    float *xyz0, float *motion);
void oracle_disparity(const uint8_t *l, const uint8_t *r, int H, int W, int pitch, int D, int P1, int P2,
                      unsigned mask, int tol, int16_t *w, float *disp, uint8_t *valid);
void oracle_disparity_ex(const uint8_t *l, const uint8_t *r, int H, int W, int pitch, int D, int P1, int P2,
                         unsigned mask, int tol, int flags, int16_t *w, float *disp, uint8_t *valid);
void oracle_densify(const float *sf4, const uint8_t *valid, int H, int W, float *out, uint8_t *fill);
void oracle_temporal_check(const float *a, const uint8_t *va, const float *b, const uint8_t *vb, int H, int W,
                           float tau_f, float tau_d, uint8_t *out);
void oracle_aggregate_at(const uint64_t *cb, const uint64_t *cm, int H, int W, int D, int right, int P1, int P2,
                         unsigned mask, int x, int y, uint16_t *S);
void oracle_disparity_at(const uint8_t *l, const uint8_t *r, int H, int W, int pitch, int D, int P1, int P2,
                         int tol, const int *xs, const int *ys, int n, int16_t *w, float *disp, uint8_t *valid);
uint64_t oracle_splitmix64(uint64_t seed, uint64_t c);
void oracle_pyr_down(const uint8_t *in, int H, int W, uint8_t *out);
int oracle_flow_cost(const uint64_t *c0, const uint64_t *c1, int H, int W, int x, int y, int fu, int fv);
void oracle_pm_offset(uint64_t seed, int level, int iter, int k, int x, int y, int r, int *ou, int *ov);
int oracle_pm_pixel(const uint64_t *c0, const uint64_t *c1, int H, int W, int level, int iter, int Rl,
                    uint64_t seed, const int16_t *fin, int x, int y, int *bu, int *bv, int *trace, int max_trace);
void oracle_pm_flow(const uint8_t *A, const uint8_t *B, int H, int W, int levels, int iters, int R,
                    int fine_radius, uint64_t seed, int16_t *flow);
void oracle_fb_check(const int16_t *F, const int16_t *B, int H, int W, int tol, float *out);
void oracle_flow(const uint8_t *L0, const uint8_t *L1, int H, int W, int levels, int iters, int R, int fine_radius,
                 uint64_t seed, int tol, int16_t *F, int16_t *B, float *out);
int oracle_lrnet_nparams(void);
float oracle_bf16(float x);
void oracle_features(const uint8_t *img, int pitch, const uint16_t *S, const int16_t *wta, int H, int W, int D,
                     int P2, float *feat);
double oracle_lrnet(const float *feat, const uint8_t *label, int B, int H, int W, const float *params,
                    int round_bf16, float *grad, float *logits);
void oracle_lrnet_backward(const float *feat, const float *dz4, int B, int H, int W, const float *params,
                           int round_bf16, float *grad);
void oracle_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1, float b2, float eps,
                 float b1t, float b2t);

static uint64_t g_state = 1801;
static uint32_t rnd(void)
{
    g_state = g_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (uint32_t)(g_state >> 33);
}
static float frnd(void) { return (float)(rnd() & 0xFFFFFF) / (float)0x1000000; }

static void stereo(int H, int W, int D)
{
    const int pitch = W + 3;
    const size_t npx = (size_t)H * W, n = npx * D;
    uint8_t *l = malloc((size_t)H * pitch), *r = malloc((size_t)H * pitch);
    for (int i = 0; i < H * pitch; ++i) {
        l[i] = (uint8_t)rnd();
        r[i] = (uint8_t)rnd();
    }
    uint64_t *cl = malloc(npx * 8), *cr = malloc(npx * 8);
    oracle_census(l, H, W, pitch, cl);
    oracle_census(r, H, W, pitch, cr);
    uint8_t *cost = malloc(n);
    int32_t *Lr = malloc(n * 4);
    uint16_t *S = malloc(n * 2), *S2 = malloc(n * 2);
    int16_t *wl = malloc(npx * 2), *wr = malloc(npx * 2);
    float *ds = malloc(npx * 4), *disp = malloc(npx * 4), *med = malloc(npx * 4);
    uint8_t *valid = malloc(npx);
    for (int right = 0; right < 2; ++right) {
        oracle_cost(right ? cr : cl, right ? cl : cr, H, W, D, right, cost);
        for (int dir = 0; dir < 8; ++dir) {
            oracle_path_cost(cost, H, W, D, 10, 120, dir, Lr);
            oracle_path_cost_adaptive(cost, l, pitch, H, W, D, 10, 120, dir, Lr);
        }
        oracle_aggregate(cost, H, W, D, 10, 120, 0xFFu, S);
        oracle_aggregate(cost, H, W, D, 0, 0, 0x0Fu, S2);
        oracle_aggregate_adaptive(cost, right ? r : l, pitch, H, W, D, 7, 8000, 0xFFu, S2);
        oracle_wta(S, H, W, D, right ? wr : wl, right ? NULL : ds);
    }
    oracle_lr_check(wl, wr, ds, H, W, 1, valid, disp);
    oracle_no_check(ds, H, W, valid, disp);
    oracle_wta_right_diag(S, H, W, D, wr);
    oracle_median3x3(ds, H, W, med);
    float *feat = malloc(npx * 16);
    oracle_features(l, pitch, S, wl, H, W, D, 120, feat);
    oracle_disparity(l, r, H, W, pitch, D, 10, 120, 0xFFu, 1, wl, disp, valid);
    for (int flags = 0; flags < 8; ++flags) oracle_disparity_ex(l, r, H, W, pitch, D, 10, 120, 0xFFu, 1, flags, wl, disp, valid);
    uint16_t *s1 = malloc((size_t)D * 2);
    oracle_aggregate_at(cl, cr, H, W, D, 0, 10, 120, 0xFFu, W - 1, H - 1, s1);
    oracle_aggregate_at(cr, cl, H, W, D, 1, 10, 120, 0xFFu, 0, 0, s1);
    int xs[3] = {0, W - 1, W / 2}, ys[3] = {0, H - 1, H / 2};
    float d3[3];
    int16_t w3[3];
    uint8_t v3[3];
    oracle_disparity_at(l, r, H, W, pitch, D, 10, 120, 1, xs, ys, 3, w3, d3, v3);
    free(s1);
    free(l); free(r); free(cl); free(cr); free(cost); free(Lr); free(S); free(S2);
    free(wl); free(wr); free(ds); free(disp); free(med); free(valid); free(feat);
}

static void scene(int H, int W)
{
    const size_t npx = (size_t)H * W;
    float *d0 = malloc(npx * 4), *d1 = malloc(npx * 4), *flow = malloc(npx * 8);
    uint8_t *v0 = malloc(npx), *v1 = malloc(npx), *valid = malloc(npx), *fill = malloc(npx), *tv = malloc(npx);
    float *sf4 = malloc(npx * 16), *sf4b = malloc(npx * 16), *xyz = malloc(npx * 12), *mot = malloc(npx * 12);
    float *dense = malloc(npx * 16);
    for (size_t i = 0; i < npx; ++i) {
        d0[i] = frnd() * 40.0f - 1.0f;
        d1[i] = frnd() * 40.0f - 1.0f;
        v0[i] = (uint8_t)(rnd() & 1);
        v1[i] = (uint8_t)(rnd() & 1);
        flow[2 * i] = (rnd() % 7 == 0) ? nanf("") : frnd() * 30.0f - 15.0f;
        flow[2 * i + 1] = frnd() * 10.0f - 5.0f;
    }
    oracle_combine(d0, v0, d1, v1, flow, H, W, 1, 721.5f, 0.54f, (W - 1) / 2.0f, (H - 1) / 2.0f, sf4, valid, xyz, mot);
    oracle_combine(d0, v0, d1, v1, flow, H, W, 0, 0, 0, 0, 0, sf4b, valid, xyz, mot);
    oracle_densify(sf4, valid, H, W, dense, fill);
    oracle_temporal_check(sf4, valid, sf4, valid, H, W, 2.0f, 1.0f, tv);
    free(d0); free(d1); free(flow); free(v0); free(v1); free(valid); free(fill); free(tv);
    free(sf4); free(sf4b); free(xyz); free(mot); free(dense);
}

static void flowcase(int H, int W)
{
    const size_t npx = (size_t)H * W;
    uint8_t *a = malloc(npx), *b = malloc(npx);
    for (size_t i = 0; i < npx; ++i) {
        a[i] = (uint8_t)rnd();
        b[i] = (uint8_t)rnd();
    }
    uint8_t *p = malloc(((H + 1) / 2) * (size_t)((W + 1) / 2));
    oracle_pyr_down(a, H, W, p);
    uint64_t *c0 = malloc(npx * 8), *c1 = malloc(npx * 8);
    oracle_census(a, H, W, W, c0);
    oracle_census(b, H, W, W, c1);
    (void)oracle_flow_cost(c0, c1, H, W, 0, 0, W - 1, H - 1);
    (void)oracle_flow_cost(c0, c1, H, W, W - 1, H - 1, 1, 1);
    int16_t *F = calloc(npx * 2, 2), *B = calloc(npx * 2, 2);
    int tr[3 * 32], bu, bv, ou, ov;
    oracle_pm_offset(7, 3, 5, 2, W - 1, H - 1, 9, &ou, &ov);
    (void)oracle_pm_pixel(c0, c1, H, W, 0, 0, 16, 7, F, W - 1, H - 1, &bu, &bv, tr, 32);
    (void)oracle_pm_pixel(c0, c1, H, W, 0, 0, 16, 7, F, 0, 0, &bu, &bv, NULL, 0);
    float *out = malloc(npx * 8);
    oracle_flow(a, b, H, W, 3, 2, 16, 4, 1801, 1, F, B, out);
    oracle_fb_check(F, B, H, W, 1, out);
    free(a); free(b); free(p); free(c0); free(c1); free(F); free(B); free(out);
}

static void network(int Bn, int H, int W)
{
    const int np = oracle_lrnet_nparams();
    const size_t npx = (size_t)Bn * H * W;
    float *prm = malloc((size_t)np * 4), *g = malloc((size_t)np * 4), *m = calloc(np, 4), *v = calloc(np, 4);
    float *feat = malloc(npx * 16), *lg = malloc(npx * 4), *dz = malloc(npx * 4);
    uint8_t *lab = malloc(npx);
    for (int i = 0; i < np; ++i) prm[i] = frnd() - 0.5f;
    for (size_t i = 0; i < npx * 4; ++i) feat[i] = frnd() * 2.0f;
    for (size_t i = 0; i < npx; ++i) {
        lab[i] = (uint8_t)(rnd() & 1);
        dz[i] = frnd() - 0.5f;
    }
    for (int rb = 0; rb < 2; ++rb) {
        (void)oracle_lrnet(feat, lab, Bn, H, W, prm, rb, g, lg);
        (void)oracle_lrnet(feat, NULL, Bn, H, W, prm, rb, NULL, lg);
        oracle_lrnet_backward(feat, dz, Bn, H, W, prm, rb, g);
    }
    oracle_adam(prm, m, v, g, np, 1e-3f, 0.9f, 0.999f, 1e-8f, 0.9f, 0.999f);
    (void)oracle_bf16(nanf(""));
    (void)oracle_bf16(3.0e38f);
    free(prm); free(g); free(m); free(v); free(feat); free(lg); free(dz); free(lab);
}

int main(void)
{
    const int shapes[][3] = {{1, 1, 1}, {1, 1, 32}, {1, 9, 8}, {7, 1, 16}, {5, 11, 3}, {13, 29, 32}, {24, 40, 64}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s) stereo(shapes[s][0], shapes[s][1], shapes[s][2]);
    const int sc[][2] = {{1, 1}, {1, 7}, {6, 1}, {17, 23}};
    for (size_t s = 0; s < sizeof(sc) / sizeof(sc[0]); ++s) scene(sc[s][0], sc[s][1]);
    flowcase(1, 1);
    flowcase(3, 5);
    flowcase(33, 47);
    network(1, 1, 1);
    network(2, 5, 7);
    (void)oracle_splitmix64(0, 0);
    puts("oracle sanitizer run: clean");
    return 0;
}
