/*
 * CPU oracle for the optical-flow stand-in.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  The product path (the HIP
 * library) never calls it and shares no code, header, table or helper with it.
 *
 * The paper takes its flow from Flow Fields+ (Sec. 3.2): matches are found on
 * a coarse level first, propagated to neighbours and refined by random search
 * under a patch data term, lifted level by level to full resolution, and
 * filtered by consistency with the inverse flow.  This stand-in follows that
 * outline with choices of its own (Flow Fields+' feature initialisation and
 * the EpicFlow interpolation are not part of it):
 *   - pyramid: level l+1 is the 2x2 box mean of level l, (a+b+c+d+2)/4 in
 *     integers, odd borders clamped; level sizes ceil(W/2), ceil(H/2);
 *   - data term: at each level the 9x7 census of both images (the same census
 *     as the stereo cost); the cost of integer flow f at pixel x is the sum of
 *     the Hamming distances of the census at x + o and x + f + o for the nine
 *     offsets o in {-2, 0, 2}^2, coordinates clamped to the image; a flow
 *     whose target x + f lies outside the image is not a candidate;
 *   - start: f = 0 on the coarsest level; at a finer level f(x, y) = 2 f(x/2,
 *     y/2) of the coarser result, its target clamped into the image;
 *   - each iteration updates every pixel from the previous iteration's field
 *     (all pixels in parallel).  Candidates, in this order: the pixel's own f;
 *     the f of its neighbours at distance 1 then 4 (left, right, up, down);
 *     then random search around the best candidate so far with radius
 *     r_k = R_l >> k for k = 0, 1, ... while r_k >= 1, where R_l = max(1,
 *     R >> l) for a full-resolution range R, capped at fine_radius on every
 *     level but the coarsest when fine_radius > 0.  The lowest cost wins; the first
 *     in this order on ties;
 *   - random offsets: h = SplitMix64 output for counter c (the generator's
 *     finaliser applied to seed + (c + 1) * 0x9e3779b97f4a7c15) with
 *     c = (((level * 64 + iter) * 64 + k) * 65536 + y/8) * 65536 + x/8, so
 *     the pixels of one 8x8 tile share the offset (each still searches around
 *     its own best flow); the offset is ((h & 0xFFFF) mod (2r+1)) - r
 *     horizontally and (((h >> 16) & 0xFFFF) mod (2r+1)) - r vertically.
 *     Sec. 3.2 names random search but not its distribution: this definition
 *     gives every pixel a candidate spread over the (2r+1)^2 box around its
 *     own best flow (up to the 16-bit modulo bias), and draws one displacement
 *     per tile, so that neighbouring pixels try the same relative move of
 *     their own matches.  Per-pixel draws would be an equally valid choice;
 *     this one is fixed here and the kernels follow it;
 *   - consistency: forward flow F at x is kept iff the backward flow B (the
 *     same method from the second image to the first, with seed
 *     seed ^ 0x5bd1e995) at x' = x + F(x)
 *     satisfies |F_u(x) + B_u(x')| <= tol and |F_v(x) + B_v(x')| <= tol.
 * Plain nested loops in the order of the definitions; integer arithmetic only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void oracle_census(const uint8_t *img, int H, int W, int pitch, uint64_t *out);

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output for counter c. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

void oracle_pyr_down(const uint8_t *in, int H, int W, uint8_t *out)
{
    const int h = (H + 1) / 2, w = (W + 1) / 2;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int x0 = 2 * x, y0 = 2 * y;
            int x1 = x0 + 1 < W ? x0 + 1 : W - 1, y1 = y0 + 1 < H ? y0 + 1 : H - 1;
            int s = in[(size_t)y0 * W + x0] + in[(size_t)y0 * W + x1] + in[(size_t)y1 * W + x0] +
                    in[(size_t)y1 * W + x1];
            out[(size_t)y * w + x] = (uint8_t)((s + 2) / 4);
        }
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int popcount64(uint64_t v)
{
    int n = 0;
    while (v) {
        v &= v - 1;
        ++n;
    }
    return n;
}

/* Cost of integer flow (fu, fv) at (x, y); -1 if the target leaves the image. */
int oracle_flow_cost(const uint64_t *c0, const uint64_t *c1, int H, int W, int x, int y, int fu,
                     int fv)
{
    const int tx = x + fu, ty = y + fv;
    if (tx < 0 || tx > W - 1 || ty < 0 || ty > H - 1) return -1;
    int s = 0;
    for (int j = -2; j <= 2; j += 2)
        for (int i = -2; i <= 2; i += 2) {
            uint64_t a = c0[(size_t)clampi(y + j, 0, H - 1) * W + clampi(x + i, 0, W - 1)];
            uint64_t b = c1[(size_t)clampi(ty + j, 0, H - 1) * W + clampi(tx + i, 0, W - 1)];
            s += popcount64(a ^ b);
        }
    return s;
}

/* Random-search offset of candidate k (radius r) at pixel (x, y) of the given
 * level and iteration: the counter packs (level, iteration, k, tile row, tile
 * column) with the 8x8 tile of the pixel; the low 16 bits of the generator's
 * output give the horizontal offset, the next 16 bits the vertical one. */
void oracle_pm_offset(uint64_t seed, int level, int iter, int k, int x, int y, int r, int *ou, int *ov)
{
    const uint64_t ctr =
        ((((uint64_t)level * 64 + (uint64_t)iter) * 64 + (uint64_t)k) * 65536 + (uint64_t)(y / 8)) * 65536 +
        (uint64_t)(x / 8);
    const uint64_t h = oracle_splitmix64(seed, ctr);
    *ou = (int)((h & 0xFFFFu) % (uint64_t)(2 * r + 1)) - r;
    *ov = (int)(((h >> 16) & 0xFFFFu) % (uint64_t)(2 * r + 1)) - r;
}

/* One pixel of one iteration: evaluates the candidates in their order and
 * returns how many it evaluated; *bu, *bv receive the winner.  When trace is
 * not NULL, candidate n is recorded as trace[3n .. 3n+2] = (u, v, cost) for
 * the first max_trace candidates (cost -1: target outside the image). */
int oracle_pm_pixel(const uint64_t *c0, const uint64_t *c1, int H, int W, int level, int iter, int Rl,
                    uint64_t seed, const int16_t *fin, int x, int y, int *bu_out, int *bv_out, int *trace,
                    int max_trace)
{
    const int du[4] = {-1, +1, 0, 0}, dv[4] = {0, 0, -1, +1};
    const int dist[2] = {1, 4};
    int n = 0;
#define PM_RECORD(U, V, C)                  \
    do {                                    \
        if (trace && n < max_trace) {       \
            trace[3 * n] = (U);             \
            trace[3 * n + 1] = (V);         \
            trace[3 * n + 2] = (C);         \
        }                                   \
        ++n;                                \
    } while (0)
    const size_t i = (size_t)y * W + x;
    int bu = fin[2 * i], bv = fin[2 * i + 1];
    int best = oracle_flow_cost(c0, c1, H, W, x, y, bu, bv);
    PM_RECORD(bu, bv, best);
    if (best < 0) best = 1 << 30; /* cannot happen: fields keep targets inside */
    for (int s = 0; s < 2; ++s)
        for (int m = 0; m < 4; ++m) {
            const int nx = x + dist[s] * du[m], ny = y + dist[s] * dv[m];
            if (nx < 0 || nx > W - 1 || ny < 0 || ny > H - 1) continue;
            const size_t k = (size_t)ny * W + nx;
            const int cu = fin[2 * k], cv = fin[2 * k + 1];
            const int c = oracle_flow_cost(c0, c1, H, W, x, y, cu, cv);
            PM_RECORD(cu, cv, c);
            if (c >= 0 && c < best) {
                best = c;
                bu = cu;
                bv = cv;
            }
        }
    for (int k = 0; (Rl >> k) >= 1; ++k) {
        int ou, ov;
        oracle_pm_offset(seed, level, iter, k, x, y, Rl >> k, &ou, &ov);
        const int cu = bu + ou, cv = bv + ov;
        const int c = oracle_flow_cost(c0, c1, H, W, x, y, cu, cv);
        PM_RECORD(cu, cv, c);
        if (c >= 0 && c < best) {
            best = c;
            bu = cu;
            bv = cv;
        }
    }
#undef PM_RECORD
    *bu_out = bu;
    *bv_out = bv;
    return n;
}

/* One iteration on one level: flow_in / flow_out [H][W][2] int16. */
static void pm_iteration(const uint64_t *c0, const uint64_t *c1, int H, int W, int level, int iter,
                         int Rl, uint64_t seed, const int16_t *fin, int16_t *fout)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t i = (size_t)y * W + x;
            int bu, bv;
            oracle_pm_pixel(c0, c1, H, W, level, iter, Rl, seed, fin, x, y, &bu, &bv, NULL, 0);
            fout[2 * i] = (int16_t)bu;
            fout[2 * i + 1] = (int16_t)bv;
        }
}

/* Integer flow from image A to image B ([H][W] uint8, pitch W): levels >= 1,
 * iters >= 1 per level, R >= 1 the full-resolution search range.  flow
 * [H][W][2] int16 (output). */
void oracle_pm_flow(const uint8_t *A, const uint8_t *B, int H, int W, int levels, int iters, int R,
                    int fine_radius, uint64_t seed, int16_t *flow)
{
    uint8_t *pa[16], *pb[16];
    int hs[16], ws[16];
    hs[0] = H;
    ws[0] = W;
    pa[0] = (uint8_t *)malloc((size_t)H * W);
    pb[0] = (uint8_t *)malloc((size_t)H * W);
    memcpy(pa[0], A, (size_t)H * W);
    memcpy(pb[0], B, (size_t)H * W);
    for (int l = 1; l < levels; ++l) {
        hs[l] = (hs[l - 1] + 1) / 2;
        ws[l] = (ws[l - 1] + 1) / 2;
        pa[l] = (uint8_t *)malloc((size_t)hs[l] * ws[l]);
        pb[l] = (uint8_t *)malloc((size_t)hs[l] * ws[l]);
        oracle_pyr_down(pa[l - 1], hs[l - 1], ws[l - 1], pa[l]);
        oracle_pyr_down(pb[l - 1], hs[l - 1], ws[l - 1], pb[l]);
    }
    int16_t *cur = NULL;
    for (int l = levels - 1; l >= 0; --l) {
        const int h = hs[l], w = ws[l];
        uint64_t *c0 = (uint64_t *)malloc((size_t)h * w * 8), *c1 = (uint64_t *)malloc((size_t)h * w * 8);
        oracle_census(pa[l], h, w, w, c0);
        oracle_census(pb[l], h, w, w, c1);
        int16_t *f = (int16_t *)calloc((size_t)h * w * 2, sizeof(int16_t));
        if (cur) {
            const int hc = hs[l + 1], wc = ws[l + 1];
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < w; ++x) {
                    const size_t k = (size_t)clampi(y / 2, 0, hc - 1) * wc + clampi(x / 2, 0, wc - 1);
                    const int fu = 2 * cur[2 * k], fv = 2 * cur[2 * k + 1];
                    f[2 * ((size_t)y * w + x)] = (int16_t)(clampi(x + fu, 0, w - 1) - x);
                    f[2 * ((size_t)y * w + x) + 1] = (int16_t)(clampi(y + fv, 0, h - 1) - y);
                }
            free(cur);
        }
        int16_t *g = (int16_t *)malloc((size_t)h * w * 2 * sizeof(int16_t));
        int Rl = (R >> l) > 1 ? (R >> l) : 1;
        if (l < levels - 1 && fine_radius > 0 && Rl > fine_radius) Rl = fine_radius;
        for (int it = 0; it < iters; ++it) {
            pm_iteration(c0, c1, h, w, l, it, Rl, seed, f, g);
            int16_t *t = f;
            f = g;
            g = t;
        }
        free(g);
        free(c0);
        free(c1);
        cur = f;
    }
    memcpy(flow, cur, (size_t)H * W * 2 * sizeof(int16_t));
    free(cur);
    for (int l = 0; l < levels; ++l) {
        free(pa[l]);
        free(pb[l]);
    }
}

/* Forward-backward consistency: out [H][W][2] float = F where kept, NaN else. */
void oracle_fb_check(const int16_t *F, const int16_t *B, int H, int W, int tol, float *out)
{
    const float nanv = nanf("");
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t i = (size_t)y * W + x;
            const int fu = F[2 * i], fv = F[2 * i + 1];
            const int tx = x + fu, ty = y + fv;
            int ok = 0;
            if (tx >= 0 && tx < W && ty >= 0 && ty < H) {
                const size_t k = (size_t)ty * W + tx;
                const int eu = fu + B[2 * k], ev = fv + B[2 * k + 1];
                ok = (eu >= -tol && eu <= tol && ev >= -tol && ev <= tol);
            }
            out[2 * i] = ok ? (float)fu : nanv;
            out[2 * i + 1] = ok ? (float)fv : nanv;
        }
}

/* The whole stand-in: forward and backward integer flows, then the check. */
void oracle_flow(const uint8_t *L0, const uint8_t *L1, int H, int W, int levels, int iters, int R,
                 int fine_radius, uint64_t seed, int tol, int16_t *F, int16_t *B, float *out)
{
    oracle_pm_flow(L0, L1, H, W, levels, iters, R, fine_radius, seed, F);
    oracle_pm_flow(L1, L0, H, W, levels, iters, R, fine_radius, seed ^ 0x5bd1e995ULL, B);
    oracle_fb_check(F, B, H, W, tol, out);
}
