/*
 * CPU oracle for the stereo / scene-flow hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  The product path (the HIP
 * library) never calls it, shares no code, header, table or helper with it,
 * and must fail loudly when its own extension is missing.
 *
 * Everything here is plain, single-threaded C written for readability: nested
 * loops in the order the definitions are stated, no blocking, no fusion, no
 * SIMD intrinsics, no threads.  Integer stages are exact; FP32 stages perform
 * the stated operations in the stated order (build with -ffp-contract=off).
 *
 * Sources of each definition:
 *   - Paper, Sec. 3.1 (Eq. 1): the disparity map D: Omega -> R+, computed by
 *     semi-global matching over eight paths radiating from each pixel, with a
 *     left-right consistency check that removes inconsistent pixels.
 *   - Paper, Sec. 3.3 (scene-flow map S: Omega -> R^4, its case definition
 *     and the bilinear interpolation equation), and the remark that the
 *     disparity difference gives the motion along the viewing direction.
 *   - The cited SGM method (Hirschmueller, PAMI 2008) for the path-cost
 *     recurrence with penalties P1 / P2.
 *   - The workload definition for what the paper leaves open: 9x7 census,
 *     Hamming cost, D disparities, P1 = 10, P2 = 120, LR tolerance 1 px,
 *     parabolic sub-pixel refinement, f = 721.5 px, B = 0.54 m.
 * Readings of points the paper leaves open are listed next to each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_CMAX 62 /* 62-bit census descriptor => Hamming cost in [0, 62] */

/* ------------------------------------------------------------------------ */
/* Census transform (matching cost of Sec. 3.1; the paper names none).
 * Reading: 9 wide (dx = -4..4) by 7 tall (dy = -3..3) window, neighbours in
 * row-major order with the centre skipped; each neighbour contributes one bit,
 * 1 iff neighbour < centre; the first neighbour ends up in bit 61, the last in
 * bit 0; window pixels outside the image take the nearest edge pixel. */
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

void oracle_census(const uint8_t *img, int H, int W, int pitch, uint64_t *out)
{
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            uint8_t centre = img[(size_t)y * pitch + x];
            uint64_t code = 0;
            for (int dy = -3; dy <= 3; ++dy) {
                for (int dx = -4; dx <= 4; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    int yy = clampi(y + dy, 0, H - 1);
                    int xx = clampi(x + dx, 0, W - 1);
                    uint8_t nb = img[(size_t)yy * pitch + xx];
                    code = (code << 1) | (uint64_t)(nb < centre ? 1 : 0);
                }
            }
            out[(size_t)y * W + x] = code;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Matching cost: Hamming distance between the base pixel's descriptor and the
 * match pixel's, one disparity hypothesis d in [0, D) at a time.
 *   base = left : match pixel (x - d, y); base = right: match pixel (x + d, y).
 * Reading: a match pixel outside the image costs the maximum, 62.
 * Layout: cost[(y * W + x) * D + d]. */
static int popcount64(uint64_t v)
{
    int n = 0;
    while (v) { n += (int)(v & 1u); v >>= 1; }
    return n;
}

void oracle_cost(const uint64_t *cen_base, const uint64_t *cen_match, int H, int W, int D,
                 int base_is_right, uint8_t *cost)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int d = 0; d < D; ++d) {
                int xm = base_is_right ? x + d : x - d;
                int c;
                if (xm < 0 || xm > W - 1)
                    c = ORACLE_CMAX;
                else
                    c = popcount64(cen_base[(size_t)y * W + x] ^ cen_match[(size_t)y * W + xm]);
                cost[((size_t)y * W + x) * D + d] = (uint8_t)c;
            }
}

/* ------------------------------------------------------------------------ */
/* Path costs and their sum (Sec. 3.1: eight paths radiating from each pixel;
 * recurrence of the cited SGM method).  For direction r the predecessor of p
 * is p - r.  If p - r lies outside the image, Lr(p, d) = C(p, d); otherwise,
 * with M = min_k Lr(p - r, k),
 *   Lr(p, d) = C(p, d) + min(Lr(p-r, d), Lr(p-r, d-1) + P1, Lr(p-r, d+1) + P1,
 *                            M + P2) - M,
 * where terms with d - 1 or d + 1 outside [0, D) are left out.
 * Direction numbering (r = (rx, ry)):
 *   0:(+1,0) 1:(-1,0) 2:(0,+1) 3:(0,-1) 4:(+1,+1) 5:(-1,+1) 6:(+1,-1) 7:(-1,-1)
 * S(p, d) = sum of Lr(p, d) over the directions whose bit is set in path_mask.
 * Exact integers; requires P2 >= P1. */
static const int ORACLE_DIR[8][2] = {
    {+1, 0}, {-1, 0}, {0, +1}, {0, -1}, {+1, +1}, {-1, +1}, {+1, -1}, {-1, -1}};

/* One direction's path cost volume, Lr[(y * W + x) * D + d]. */
/* Path cost of one direction with the large-jump penalty taken per pixel:
 * p2map == NULL gives the constant P2; otherwise the penalty at p is
 * p2map(p, p - r) (see oracle_path_cost_adaptive). */
static int adaptive_p2(const uint8_t *img, int pitch, int x, int y, int px, int py, int P1, int P2)
{
    int g = (int)img[(size_t)y * pitch + x] - (int)img[(size_t)py * pitch + px];
    if (g < 0) g = -g;
    if (g == 0) return P2;
    int q = P2 / g;
    return q > P1 ? q : P1;
}

static void path_cost(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W, int D,
                      int P1, int P2, int dir, int32_t *Lr)
{
    int rx = ORACLE_DIR[dir][0], ry = ORACLE_DIR[dir][1];
    /* Visit pixels so that p - r is always visited before p. */
    for (int iy = 0; iy < H; ++iy) {
        int y = (ry >= 0) ? iy : H - 1 - iy;
        for (int ix = 0; ix < W; ++ix) {
            int x = (rx >= 0) ? ix : W - 1 - ix;
            const uint8_t *C = cost + ((size_t)y * W + x) * D;
            int32_t *L = Lr + ((size_t)y * W + x) * D;
            int px = x - rx, py = y - ry;
            if (px < 0 || px > W - 1 || py < 0 || py > H - 1) {
                for (int d = 0; d < D; ++d) L[d] = C[d];
                continue;
            }
            const int p2 = img ? adaptive_p2(img, pitch, x, y, px, py, P1, P2) : P2;
            const int32_t *Lp = Lr + ((size_t)py * W + px) * D;
            int32_t M = Lp[0];
            for (int k = 1; k < D; ++k)
                if (Lp[k] < M) M = Lp[k];
            for (int d = 0; d < D; ++d) {
                int32_t best = Lp[d];
                if (d - 1 >= 0 && Lp[d - 1] + P1 < best) best = Lp[d - 1] + P1;
                if (d + 1 <= D - 1 && Lp[d + 1] + P1 < best) best = Lp[d + 1] + P1;
                if (M + p2 < best) best = M + p2;
                L[d] = (int32_t)C[d] + best - M;
            }
        }
    }
}

void oracle_path_cost(const uint8_t *cost, int H, int W, int D, int P1, int P2, int dir,
                      int32_t *Lr)
{
    path_cost(cost, NULL, 0, H, W, D, P1, P2, dir, Lr);
}

static void aggregate(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W, int D,
                      int P1, int P2, unsigned path_mask, uint16_t *S)
{
    size_t n = (size_t)H * W * D;
    int32_t *Lr = (int32_t *)malloc(n * sizeof(int32_t));
    int32_t *acc = (int32_t *)calloc(n, sizeof(int32_t));
    for (int r = 0; r < 8; ++r) {
        if (!(path_mask & (1u << r))) continue;
        path_cost(cost, img, pitch, H, W, D, P1, P2, r, Lr);
        for (size_t i = 0; i < n; ++i) acc[i] += Lr[i];
    }
    for (size_t i = 0; i < n; ++i) S[i] = (uint16_t)acc[i];
    free(Lr);
    free(acc);
}

void oracle_aggregate(const uint8_t *cost, int H, int W, int D, int P1, int P2,
                      unsigned path_mask, uint16_t *S)
{
    aggregate(cost, NULL, 0, H, W, D, P1, P2, path_mask, S);
}

/* Intensity-adaptive large-jump penalty (a variant of the cited SGM method:
 * the penalty for a disparity jump of more than one step is lowered across
 * intensity edges of the base image).  Reading: at pixel p with predecessor
 * p - r on the path, g = |I(p) - I(p - r)| on the base image; the penalty is
 * P2 if g = 0, else max(P1, floor(P2 / g)).  Path starts have no predecessor
 * (Lr = C there), so no penalty applies.  img is [H][pitch] uint8. */
void oracle_path_cost_adaptive(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W,
                               int D, int P1, int P2, int dir, int32_t *Lr)
{
    path_cost(cost, img, pitch, H, W, D, P1, P2, dir, Lr);
}

void oracle_aggregate_adaptive(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W,
                               int D, int P1, int P2, unsigned path_mask, uint16_t *S)
{
    aggregate(cost, img, pitch, H, W, D, P1, P2, path_mask, S);
}

/* ------------------------------------------------------------------------ */
/* Winner-take-all with parabolic sub-pixel refinement (the map D of Eq. 1 is
 * real valued).  Reading: d* = smallest d reaching min_k S(p, k); if
 * 0 < d* < D - 1 and den = S(d*-1) - 2 S(d*) + S(d*+1) > 0, then
 * d_sub = d* + (S(d*-1) - S(d*+1)) / (2 den), one FP32 division then one FP32
 * addition; otherwise d_sub = d*. */
void oracle_wta(const uint16_t *S, int H, int W, int D, int16_t *wta, float *dsub)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const uint16_t *s = S + ((size_t)y * W + x) * D;
            int best = 0;
            for (int d = 1; d < D; ++d)
                if (s[d] < s[best]) best = d;
            float sub = (float)best;
            if (best > 0 && best < D - 1) {
                int a = s[best - 1], b = s[best], c = s[best + 1];
                int den = a - 2 * b + c;
                if (den > 0) {
                    float off = (float)(a - c) / (float)(2 * den);
                    sub = (float)best + off;
                }
            }
            wta[(size_t)y * W + x] = (int16_t)best;
            if (dsub) dsub[(size_t)y * W + x] = sub;
        }
}

/* ------------------------------------------------------------------------ */
/* Left-right consistency check (Sec. 3.1: compare the two computed disparity
 * maps and remove inconsistent pixels, which makes the map non-dense).
 * Reading: compared on integer WTA disparities; left pixel (x, y) is valid iff
 * q = x - d*_L >= 0 and |d*_L(x, y) - d*_R(q, y)| <= tol.  The output map holds
 * d_sub where valid and -1.0f elsewhere; the uint8 mask is authoritative. */
void oracle_lr_check(const int16_t *wtaL, const int16_t *wtaR, const float *dsubL, int H, int W,
                     int tol, uint8_t *valid, float *disp)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int dl = wtaL[(size_t)y * W + x];
            int q = x - dl;
            int ok = 0;
            if (q >= 0) {
                int dr = wtaR[(size_t)y * W + q];
                int diff = dl - dr;
                if (diff < 0) diff = -diff;
                ok = diff <= tol;
            }
            valid[(size_t)y * W + x] = (uint8_t)ok;
            disp[(size_t)y * W + x] = ok ? dsubL[(size_t)y * W + x] : -1.0f;
        }
}

/* Without a right view every pixel is kept (valid := 1, disp := d_sub). */
void oracle_no_check(const float *dsubL, int H, int W, uint8_t *valid, float *disp)
{
    for (size_t i = 0; i < (size_t)H * W; ++i) {
        valid[i] = 1;
        disp[i] = dsubL[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Right-view disparity without a second aggregation (a variant of the cited
 * SGM method: the match image's disparity at q lies on the diagonal of the
 * base volume).  Reading: for right pixel (q, y), d*_R is the smallest d in
 * [0, D) with q + d <= W - 1 that reaches the minimum of S_L(q + d, y, d) over
 * those d. */
void oracle_wta_right_diag(const uint16_t *S, int H, int W, int D, int16_t *wtaR)
{
    for (int y = 0; y < H; ++y)
        for (int q = 0; q < W; ++q) {
            int best = 0;
            unsigned bestv = S[((size_t)y * W + q) * D + 0];
            for (int d = 1; d < D && q + d <= W - 1; ++d) {
                unsigned v = S[((size_t)y * W + (q + d)) * D + d];
                if (v < bestv) {
                    bestv = v;
                    best = d;
                }
            }
            wtaR[(size_t)y * W + q] = (int16_t)best;
        }
}

/* 3x3 median filter (the cited method's post-filter of the disparity image).
 * Reading: out(x, y) = the fifth smallest of the nine values at (x + i, y + j),
 * i, j in {-1, 0, 1}, with coordinates clamped to the image; it is applied to
 * the dense sub-pixel map, before the LR mask. */
void oracle_median3x3(const float *in, int H, int W, float *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            float v[9];
            int n = 0;
            for (int j = -1; j <= 1; ++j)
                for (int i = -1; i <= 1; ++i)
                    v[n++] = in[(size_t)clampi(y + j, 0, H - 1) * W + clampi(x + i, 0, W - 1)];
            for (int a = 1; a < 9; ++a) { /* insertion sort */
                float t = v[a];
                int b = a - 1;
                while (b >= 0 && v[b] > t) {
                    v[b + 1] = v[b];
                    --b;
                }
                v[b + 1] = t;
            }
            out[(size_t)y * W + x] = v[4];
        }
}

/* ------------------------------------------------------------------------ */
/* Combination (Sec. 3.3).  S(x) = (u, v, d0, d1) with (u, v) = F(x),
 * d0 = D0(x), d1 = D1(x + F(x)) read by the bilinear equation; S(x) is
 * undefined unless x and x' = x + F(x) are in Omega and D0(x), D1(x') are
 * valid.  Readings:
 *   - x' is in Omega iff 0 <= x' <= W-1 and 0 <= y' <= H-1 (a NaN fails);
 *   - x0 = floor(x'), y0 = floor(y'), the "+1" taps are clamped to the last
 *     row / column (where their weight is 0), and D1(x') counts as valid iff
 *     all four taps are valid;
 *   - the four bilinear terms are summed in the printed order, left to right,
 *     each term as (D * w1) * w2, in FP32.
 * Triangulation (Sec. 3.3: the four values plus the camera fully describe 3-D
 * geometry and motion; the disparity change gives the motion along the view
 * direction).  Reading: pinhole model with focal length f, baseline B and
 * principal point (cx, cy); Z = (f*B)/d with f*B formed once in FP32,
 * X = ((x - cx) * Z) / f, Y = ((y - cy) * Z) / f.  P0 comes from (x, y, d0),
 * P1 from (x', y', d1) and motion = P1 - P0, defined only where S is defined
 * and d0 > 0 and d1 > 0.
 * Outputs: sf4[(y*W+x)*4 + {u, v, d0, d1}] or four NaNs; valid bit 0 = S
 * defined, bit 1 = 3-D defined; xyz0 / motion [(y*W+x)*3 + {X, Y, Z}] or NaN. */
void oracle_combine(const float *disp0, const uint8_t *valid0, const float *disp1,
                    const uint8_t *valid1, const float *flow, int H, int W, int has_cam, float f,
                    float B, float cx, float cy, float *sf4, uint8_t *valid, float *xyz0,
                    float *motion)
{
    float nanv = nanf("");
    float fB = f * B;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            float u = flow[2 * i + 0];
            float v = flow[2 * i + 1];
            float xp = (float)x + u;
            float yp = (float)y + v;
            int defined = 0;
            float d0 = 0.0f, d1 = 0.0f;
            if (valid0[i] && xp >= 0.0f && xp <= (float)(W - 1) && yp >= 0.0f &&
                yp <= (float)(H - 1)) {
                int x0 = (int)floorf(xp), y0 = (int)floorf(yp);
                int x1 = x0 + 1 < W - 1 ? x0 + 1 : W - 1;
                int y1 = y0 + 1 < H - 1 ? y0 + 1 : H - 1;
                size_t i00 = (size_t)y0 * W + x0, i10 = (size_t)y0 * W + x1;
                size_t i01 = (size_t)y1 * W + x0, i11 = (size_t)y1 * W + x1;
                if (valid1[i00] && valid1[i10] && valid1[i01] && valid1[i11]) {
                    float fx = xp - (float)x0;
                    float fy = yp - (float)y0;
                    float t00 = (disp1[i00] * (1.0f - fx)) * (1.0f - fy);
                    float t10 = (disp1[i10] * fx) * (1.0f - fy);
                    float t01 = (disp1[i01] * (1.0f - fx)) * fy;
                    float t11 = (disp1[i11] * fx) * fy;
                    d1 = ((t00 + t10) + t01) + t11;
                    d0 = disp0[i];
                    defined = 1;
                }
            }
            uint8_t vb = 0;
            if (defined) {
                vb = 1;
                sf4[4 * i + 0] = u;
                sf4[4 * i + 1] = v;
                sf4[4 * i + 2] = d0;
                sf4[4 * i + 3] = d1;
            } else {
                for (int k = 0; k < 4; ++k) sf4[4 * i + k] = nanv;
            }
            if (has_cam) {
                if (defined && d0 > 0.0f && d1 > 0.0f) {
                    vb |= 2;
                    float Z0 = fB / d0;
                    float X0 = (((float)x - cx) * Z0) / f;
                    float Y0 = (((float)y - cy) * Z0) / f;
                    float Z1 = fB / d1;
                    float X1 = ((xp - cx) * Z1) / f;
                    float Y1 = ((yp - cy) * Z1) / f;
                    xyz0[3 * i + 0] = X0;
                    xyz0[3 * i + 1] = Y0;
                    xyz0[3 * i + 2] = Z0;
                    motion[3 * i + 0] = X1 - X0;
                    motion[3 * i + 1] = Y1 - Y0;
                    motion[3 * i + 2] = Z1 - Z0;
                } else {
                    for (int k = 0; k < 3; ++k) {
                        xyz0[3 * i + k] = nanv;
                        motion[3 * i + k] = nanv;
                    }
                }
            }
            valid[i] = vb;
        }
}

/* ------------------------------------------------------------------------ */
/* Whole plain disparity map for one stereo pair: census of both views, left
 * and right cost volumes, 8-path aggregation of each, WTA + sub-pixel of each,
 * LR check.  Convenience wrapper over the functions above for the CPU
 * baseline; S volumes are allocated here. */
void oracle_disparity(const uint8_t *left, const uint8_t *right, int H, int W, int pitch, int D,
                      int P1, int P2, unsigned path_mask, int tol, int16_t *wtaL, float *disp,
                      uint8_t *valid)
{
    size_t npx = (size_t)H * W, n = npx * D;
    uint64_t *cl = (uint64_t *)malloc(npx * 8), *cr = (uint64_t *)malloc(npx * 8);
    uint8_t *cost = (uint8_t *)malloc(n);
    uint16_t *S = (uint16_t *)malloc(n * 2);
    int16_t *wtaR = (int16_t *)malloc(npx * 2);
    float *dsubL = (float *)malloc(npx * 4);
    oracle_census(left, H, W, pitch, cl);
    oracle_census(right, H, W, pitch, cr);
    oracle_cost(cr, cl, H, W, D, 1, cost);
    oracle_aggregate(cost, H, W, D, P1, P2, path_mask, S);
    oracle_wta(S, H, W, D, wtaR, NULL);
    oracle_cost(cl, cr, H, W, D, 0, cost);
    oracle_aggregate(cost, H, W, D, P1, P2, path_mask, S);
    oracle_wta(S, H, W, D, wtaL, dsubL);
    oracle_lr_check(wtaL, wtaR, dsubL, H, W, tol, valid, disp);
    free(cl); free(cr); free(cost); free(S); free(wtaR); free(dsubL);
}

/* The same with the variants: flags bit 0 = right map by the diagonal search
 * in S_L (no right-view aggregation), bit 1 = 3x3 median of the left sub-pixel
 * map before the LR mask, bit 2 = intensity-adaptive P2 (each view's base
 * image: the left image for the left view, the right image for the right). */
void oracle_disparity_ex(const uint8_t *left, const uint8_t *right, int H, int W, int pitch, int D,
                         int P1, int P2, unsigned path_mask, int tol, int flags, int16_t *wtaL,
                         float *disp, uint8_t *valid)
{
    size_t npx = (size_t)H * W, n = npx * D;
    uint64_t *cl = (uint64_t *)malloc(npx * 8), *cr = (uint64_t *)malloc(npx * 8);
    uint8_t *cost = (uint8_t *)malloc(n);
    uint16_t *S = (uint16_t *)malloc(n * 2);
    int16_t *wtaR = (int16_t *)malloc(npx * 2);
    float *dsubL = (float *)malloc(npx * 4), *med = (float *)malloc(npx * 4);
    const int adaptive = (flags & 4) != 0;
    oracle_census(left, H, W, pitch, cl);
    oracle_census(right, H, W, pitch, cr);
    if (!(flags & 1)) {
        oracle_cost(cr, cl, H, W, D, 1, cost);
        aggregate(cost, adaptive ? right : NULL, pitch, H, W, D, P1, P2, path_mask, S);
        oracle_wta(S, H, W, D, wtaR, NULL);
    }
    oracle_cost(cl, cr, H, W, D, 0, cost);
    aggregate(cost, adaptive ? left : NULL, pitch, H, W, D, P1, P2, path_mask, S);
    oracle_wta(S, H, W, D, wtaL, dsubL);
    if (flags & 1) oracle_wta_right_diag(S, H, W, D, wtaR);
    if (flags & 2) {
        oracle_median3x3(dsubL, H, W, med);
        memcpy(dsubL, med, npx * 4);
    }
    oracle_lr_check(wtaL, wtaR, dsubL, H, W, tol, valid, disp);
    free(cl); free(cr); free(cost); free(S); free(wtaR); free(dsubL); free(med);
}

/* ------------------------------------------------------------------------ */
/* Densification of the sparse scene-flow map (the paper reports a dense
 * version interpolated by the benchmark and names a better interpolation as
 * future work; this fill is defined here, not by the paper).
 * Reading:
 *   - an undefined pixel takes all four values (u, v, d0, d1) of the nearest
 *     defined pixel to its left or to its right in the same row; when both
 *     exist, the one with the smaller d0 (the farther surface: gaps come from
 *     occlusions and the occluded surface is the background); ties go left;
 *   - a row with no defined pixel copies, pixel by pixel, the row-filled values
 *     of the nearest row that has a defined pixel (ties go to the row above);
 *   - fill = 1 where the input was defined, 2 where filled from the row, 3 where
 *     copied from another row, 0 (and four NaNs) if no pixel is defined at all.
 * sf4 / out [H][W][4] float; valid [H][W] uint8 (bit 0 = defined). */
void oracle_densify(const float *sf4, const uint8_t *valid, int H, int W, float *out, uint8_t *fill)
{
    const float nanv = nanf("");
    int *rowok = (int *)calloc((size_t)H, sizeof(int));
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x)
            if (valid[(size_t)y * W + x] & 1) rowok[y] = 1;
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            int src = -1;
            uint8_t f = 0;
            if (valid[i] & 1) {
                src = x;
                f = 1;
            } else if (rowok[y]) {
                int xl = -1, xr = -1;
                for (int k = x - 1; k >= 0; --k)
                    if (valid[(size_t)y * W + k] & 1) { xl = k; break; }
                for (int k = x + 1; k < W; ++k)
                    if (valid[(size_t)y * W + k] & 1) { xr = k; break; }
                if (xl >= 0 && xr >= 0)
                    src = (sf4[((size_t)y * W + xr) * 4 + 2] < sf4[((size_t)y * W + xl) * 4 + 2]) ? xr : xl;
                else
                    src = xl >= 0 ? xl : xr;
                f = 2;
            }
            for (int c = 0; c < 4; ++c)
                out[i * 4 + c] = src >= 0 ? sf4[((size_t)y * W + src) * 4 + c] : nanv;
            fill[i] = f;
        }
    }
    for (int y = 0; y < H; ++y) {
        if (rowok[y]) continue;
        int best = -1;
        for (int dy = 1; dy < H && best < 0; ++dy) {
            if (y - dy >= 0 && rowok[y - dy]) best = y - dy;
            else if (y + dy < H && rowok[y + dy]) best = y + dy;
        }
        if (best < 0) continue; /* nothing defined anywhere */
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x, s = (size_t)best * W + x;
            for (int c = 0; c < 4; ++c) out[i * 4 + c] = out[s * 4 + c];
            fill[i] = 3;
        }
    }
    free(rowok);
}

/* ------------------------------------------------------------------------ */
/* Temporal validation over more than two frame pairs (the paper's future work:
 * extend the method to more frame pairs with an intermediate validation of the
 * correspondences; the rule is defined here).  With scene flow S_k between t_k
 * and t_{k+1} and S_{k+1} between t_{k+1} and t_{k+2}, pixel x is kept in S_k
 * iff
 *   - S_k(x) = (u, v, d0, d1) is defined;
 *   - q = (floor(x + u + 0.5), floor(y + v + 0.5)), the chained pixel at
 *     t_{k+1}, lies in the image and S_{k+1}(q) = (u', v', d0', d1') is
 *     defined;
 *   - |u - u'| <= tau_f, |v - v'| <= tau_f and |(d1 - d0) - (d1' - d0')| <=
 *     tau_d (motion nearly constant over the three time steps), all in FP32
 *     in this order.
 * sf4a, sf4b [H][W][4]; valid_a, valid_b [H][W] (bit 0); out [H][W] uint8. */
void oracle_temporal_check(const float *sf4a, const uint8_t *va, const float *sf4b,
                           const uint8_t *vb, int H, int W, float tau_f, float tau_d, uint8_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t i = (size_t)y * W + x;
            uint8_t ok = 0;
            if (va[i] & 1) {
                const float *a = sf4a + 4 * i;
                const float xq = floorf(((float)x + a[0]) + 0.5f);
                const float yq = floorf(((float)y + a[1]) + 0.5f);
                if (xq >= 0.0f && xq <= (float)(W - 1) && yq >= 0.0f && yq <= (float)(H - 1)) {
                    const size_t j = (size_t)yq * W + (size_t)xq;
                    if (vb[j] & 1) {
                        const float *b = sf4b + 4 * j;
                        const float ca = a[3] - a[2], cb = b[3] - b[2];
                        ok = fabsf(a[0] - b[0]) <= tau_f && fabsf(a[1] - b[1]) <= tau_f &&
                             fabsf(ca - cb) <= tau_d;
                    }
                }
            }
            out[i] = ok;
        }
}

/* ------------------------------------------------------------------------ */
/* Aggregated costs of one pixel, for checking large images at sampled pixels:
 * each direction's recurrence is run only along the line of pixels p - k r
 * (k = K .. 0, p - K r the first pixel inside the image), which is all that
 * Lr(p, .) depends on.  cen_base / cen_match [H][W]; base_is_right as in
 * oracle_cost.  S [D] uint16 (output). */
void oracle_aggregate_at(const uint64_t *cen_base, const uint64_t *cen_match, int H, int W, int D,
                         int base_is_right, int P1, int P2, unsigned path_mask, int x, int y,
                         uint16_t *S)
{
    int32_t *L = (int32_t *)malloc((size_t)D * sizeof(int32_t));
    int32_t *Ln = (int32_t *)malloc((size_t)D * sizeof(int32_t));
    int32_t *acc = (int32_t *)calloc((size_t)D, sizeof(int32_t));
    for (int r = 0; r < 8; ++r) {
        if (!(path_mask & (1u << r))) continue;
        const int rx = ORACLE_DIR[r][0], ry = ORACLE_DIR[r][1];
        int K = 0;
        while (x - (K + 1) * rx >= 0 && x - (K + 1) * rx <= W - 1 && y - (K + 1) * ry >= 0 &&
               y - (K + 1) * ry <= H - 1)
            ++K;
        for (int k = K; k >= 0; --k) {
            const int px = x - k * rx, py = y - k * ry;
            const uint64_t cb = cen_base[(size_t)py * W + px];
            int32_t M = 0;
            if (k < K) {
                M = L[0];
                for (int j = 1; j < D; ++j)
                    if (L[j] < M) M = L[j];
            }
            for (int d = 0; d < D; ++d) {
                const int mx = base_is_right ? px + d : px - d;
                const int c = (mx < 0 || mx > W - 1)
                                  ? ORACLE_CMAX
                                  : popcount64(cb ^ cen_match[(size_t)py * W + mx]);
                if (k == K) { /* the path enters the image here: Lr = C */
                    Ln[d] = c;
                    continue;
                }
                int32_t best = L[d];
                if (d - 1 >= 0 && L[d - 1] + P1 < best) best = L[d - 1] + P1;
                if (d + 1 <= D - 1 && L[d + 1] + P1 < best) best = L[d + 1] + P1;
                if (M + P2 < best) best = M + P2;
                Ln[d] = c + best - M;
            }
            memcpy(L, Ln, (size_t)D * sizeof(int32_t));
        }
        for (int d = 0; d < D; ++d) acc[d] += L[d];
    }
    for (int d = 0; d < D; ++d) S[d] = (uint16_t)acc[d];
    free(L);
    free(Ln);
    free(acc);
}

/* The plain disparity map (census, left and right aggregation, WTA, sub-pixel,
 * LR check) at n sampled pixels (xs[i], ys[i]) of one pair: the left view's
 * S at the pixel and the right view's S at q = x - d*_L.  Outputs per sample:
 * wta (d*_L), disp (d_sub or -1), valid. */
void oracle_disparity_at(const uint8_t *left, const uint8_t *right, int H, int W, int pitch, int D,
                         int P1, int P2, int tol, const int *xs, const int *ys, int n, int16_t *wta,
                         float *disp, uint8_t *valid)
{
    size_t npx = (size_t)H * W;
    uint64_t *cl = (uint64_t *)malloc(npx * 8), *cr = (uint64_t *)malloc(npx * 8);
    uint16_t *S = (uint16_t *)malloc((size_t)D * 2);
    int16_t w1[1];
    float ds[1];
    oracle_census(left, H, W, pitch, cl);
    oracle_census(right, H, W, pitch, cr);
    for (int i = 0; i < n; ++i) {
        const int x = xs[i], y = ys[i];
        oracle_aggregate_at(cl, cr, H, W, D, 0, P1, P2, 0xFFu, x, y, S);
        oracle_wta(S, 1, 1, D, w1, ds);
        const int dl = w1[0], q = x - dl;
        int ok = 0;
        if (q >= 0) {
            int16_t wr[1];
            oracle_aggregate_at(cr, cl, H, W, D, 1, P1, P2, 0xFFu, q, y, S);
            oracle_wta(S, 1, 1, D, wr, NULL);
            int diff = dl - wr[0];
            if (diff < 0) diff = -diff;
            ok = diff <= tol;
        }
        wta[i] = (int16_t)dl;
        valid[i] = (uint8_t)ok;
        disp[i] = ok ? ds[0] : -1.0f;
    }
    free(cl);
    free(cr);
    free(S);
}
