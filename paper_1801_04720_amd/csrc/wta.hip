// Winner-take-all with parabolic sub-pixel refinement, the left-right
// consistency check (paper Sec. 3.1: two computed disparity maps are compared
// and inconsistent pixels removed, leaving a non-dense map) and the per-pixel
// features of the learned stand-in for that check.
//
// One 16-lane DPP row per pixel: lane j reads disparities [4c, 4c+4) for
// c = j, j+16, ... (128 contiguous bytes per row per load), the (S, d) minimum
// is a row butterfly on the key S * 512 + d, so ties go to the smallest d.
// The frame and batch paths never write S: wta_slab_kernel sums the eight u8
// direction slabs of a pixel on the fly (one compile-time mode per launch:
// right map, left map with or without the LR check, with or without the
// network features), and wta_diag_slab_kernel adds the diagonal-search right
// map.
#include "sf_check.hpp"
#include "sf_internal.hpp"
#include "stages.hpp"

SF_CHECK_TU(wta)

namespace sf {

constexpr int WTA_NT = 256;
constexpr int WTA_PPB = WTA_NT / 16;  // pixels per block

struct WtaResult {
    uint32_t key;  // S(d*) * 512 + d*
};

__device__ __forceinline__ uint32_t s_at(const uint16_t *s, int d) { return s[d]; }

// Row-wide minimum key of one pixel's cost vector.
__device__ __forceinline__ uint32_t wta_key(const uint16_t *__restrict__ s, int D, int j)
{
    uint32_t best = 0xFFFFFFFFu;
    if ((D & 3) == 0) {
        for (int c = j; c < (D >> 2); c += 16) {
            uint2 v = reinterpret_cast<const uint2 *>(s)[c];
            const int d = 4 * c;
            best = min(best, ((v.x & 0xFFFFu) << 9) | (uint32_t)d);
            best = min(best, ((v.x >> 16) << 9) | (uint32_t)(d + 1));
            best = min(best, ((v.y & 0xFFFFu) << 9) | (uint32_t)(d + 2));
            best = min(best, ((v.y >> 16) << 9) | (uint32_t)(d + 3));
        }
    } else {
        for (int d = j; d < D; d += 16) best = min(best, ((uint32_t)s[d] << 9) | (uint32_t)d);
    }
    return row16_min(best);
}

// d* of the right view only.
__global__ __launch_bounds__(WTA_NT) void wta_right_kernel(const uint16_t *__restrict__ S, int npx,
                                                          int D, int16_t *__restrict__ wta)
{
    const int px = blockIdx.x * WTA_PPB + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    if (px >= npx) return;
    const uint32_t key = wta_key(S + (size_t)px * D, D, j);
    if (j == 0) wta[px] = (int16_t)(key & 511u);
}

__global__ __launch_bounds__(WTA_NT) void wta_left_kernel(
    const uint16_t *__restrict__ S, const int16_t *__restrict__ wta_r, const uint8_t *__restrict__ img,
    int pitch, int H, int W, int D, int P2, int tol, int16_t *__restrict__ wta,
    float *__restrict__ disp, uint8_t *__restrict__ valid, float *__restrict__ feat)
{
    const int px = blockIdx.x * WTA_PPB + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    if (px >= H * W) return;
    const uint16_t *s = S + (size_t)px * D;
    const uint32_t key = wta_key(s, D, j);
    const int ds = (int)(key & 511u);
    const uint32_t smin = key >> 9;
    uint32_t s2 = 0xFFFFFFFFu;
    if (feat) {
        // Second minimum over |d - d*| >= 2.
        for (int d = j; d < D; d += 16) {
            const int gap = d > ds ? d - ds : ds - d;
            if (gap >= 2) s2 = min(s2, (uint32_t)s[d]);
        }
        s2 = row16_min(s2);
    }
    if (j != 0) return;
    const int y = px / W, x = px - y * W;
    float sub = (float)ds;
    if (ds > 0 && ds < D - 1) {
        const int a = s[ds - 1], b = (int)smin, c = s[ds + 1];
        const int den = a - 2 * b + c;
        if (den > 0) sub = (float)ds + (float)(a - c) / (float)(2 * den);
    }
    int ok = 1;
    if (wta_r) {
        const int q = x - ds;
        ok = 0;
        if (q >= 0) {
            SF_BOUNDS(q < W && y < H, CHK_WTA_LR);
            int diff = ds - (int)wta_r[(size_t)y * W + q];
            diff = diff < 0 ? -diff : diff;
            ok = diff <= tol;
        }
    }
    wta[px] = (int16_t)ds;
    disp[px] = ok ? sub : -1.0f;
    valid[px] = (uint8_t)ok;
    if (feat) {
        if (s2 == 0xFFFFFFFFu) s2 = smin;
        float4 f;
        f.x = (float)img[(size_t)y * pitch + x] / 255.0f;
        f.y = D > 1 ? (float)ds / (float)(D - 1) : 0.0f;
        f.z = (float)smin / (float)(8 * (SF_CMAX + P2));
        f.w = (float)s2 / (float)(smin > 1 ? smin : 1u);
        reinterpret_cast<float4 *>(feat)[px] = f;
    }
}

// WTA on S = sum of u8 slabs, summed on the fly (S is never written).  Lane j
// holds slab byte positions [8c, 8c + 8), c = j and j + 16, as packed u16 sums;
// each slab load is 8 bytes per lane, 128 contiguous bytes per pixel row.  The
// aggregation stores each 16-lane chunk of K = D/16 bytes interleaved: position
// e of chunk q holds d = qK + e/2 + (e%2) K/2.
template <int K>
__device__ __forceinline__ int slab_pos_to_d(int pos)
{
    const int q = pos / K, e = pos - q * K;
    return q * K + (e >> 1) + (e & 1) * (K >> 1);
}

// The slab bytes of pixel px that lane j of a 16-lane group sums (positions
// [8c, 8c + 8), c = j and j + 16): all loads issued at once (slabs past ns
// re-read the last one; slab_add masks them to zero).
template <int K>
__device__ __forceinline__ void slab_load(const uint8_t *__restrict__ slab, size_t cells, int px, int j,
                                          int ns, u32x2 (&w)[2][8])
{
    constexpr int D = 16 * K;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = j + 16 * i;
        if (8 * c < D) {
            const uint8_t *src = slab + (size_t)px * D + 8 * c;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                w[i][k] = __builtin_nontemporal_load(
                    reinterpret_cast<const u32x2 *>(src + (size_t)min(k, ns - 1) * cells));
        }
    }
}

// Packed u16 sums of the first ns slabs from slab_load's bytes, and the
// disparity of each position.
template <int K>
__device__ __forceinline__ void slab_add(const u32x2 (&w)[2][8], int j, int ns, uint32_t (&sv)[2][4],
                                         int (&dd)[2][8])
{
    constexpr int D = 16 * K;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = j + 16 * i;
#pragma unroll
        for (int e = 0; e < 4; ++e) sv[i][e] = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) dd[i][e] = slab_pos_to_d<K>(8 * c + e);
        if (8 * c < D) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t keep = k < ns ? 0xFFFFFFFFu : 0u;
                const uint32_t lo = w[i][k].x & keep, hi = w[i][k].y & keep;
                sv[i][0] += __builtin_amdgcn_perm(0u, lo, 0x0c010c00u);
                sv[i][1] += __builtin_amdgcn_perm(0u, lo, 0x0c030c02u);
                sv[i][2] += __builtin_amdgcn_perm(0u, hi, 0x0c010c00u);
                sv[i][3] += __builtin_amdgcn_perm(0u, hi, 0x0c030c02u);
            }
        }
    }
}

// Packed u16 sums of the first ns slabs at pixel px for lane j of a 16-lane
// group (byte positions [8c, 8c + 8), c = j and j + 16), and the disparity of
// each position.  All slab loads of the lane are issued before any is used
// (slabs past ns re-read the last one and are masked to zero), so a wave keeps
// up to 16 loads in flight.
template <int K>
__device__ __forceinline__ void slab_sums(const uint8_t *__restrict__ slab, size_t cells, int px,
                                          int j, int ns, uint32_t (&sv)[2][4], int (&dd)[2][8])
{
    u32x2 w[2][8];
    slab_load<K>(slab, cells, px, j, ns, w);
    slab_add<K>(w, j, ns, sv, dd);
}

__device__ __forceinline__ uint32_t sv_val(const uint32_t (&sv)[2][4], int i, int e)
{
    return (e & 1) ? (sv[i][e >> 1] >> 16) : (sv[i][e >> 1] & 0xFFFFu);
}

// S(d* - 1), S(d* + 1) and (optionally) the minimum over |d - d*| >= 2, each
// left in every lane of the group.
template <int K, bool S2>
__device__ __forceinline__ void neighbours(const uint32_t (&sv)[2][4], const int (&dd)[2][8], int j,
                                           int ds, uint32_t &av, uint32_t &cv, uint32_t &s2)
{
    constexpr int D = 16 * K;
    av = 0;
    cv = 0;
    s2 = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = j + 16 * i;
        if (8 * c < D) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int d = dd[i][e];
                const uint32_t val = sv_val(sv, i, e);
                if (d == ds - 1) av = val;
                if (d == ds + 1) cv = val;
                if (S2) {
                    const int gap = d > ds ? d - ds : ds - d;
                    if (gap >= 2) s2 = min(s2, val);
                }
            }
        }
    }
    av = row16_max(av);
    cv = row16_max(cv);
    if (S2) s2 = row16_min(s2);
}

// Parabolic sub-pixel disparity from S(d*-1), S(d*), S(d*+1).
__device__ __forceinline__ float subpixel(int ds, int D, uint32_t av, uint32_t smin, uint32_t cv)
{
    float sub = (float)ds;
    if (ds > 0 && ds < D - 1) {
        const int den = (int)av - 2 * (int)smin + (int)cv;
        if (den > 0) sub = (float)ds + (float)((int)av - (int)cv) / (float)(2 * den);
    }
    return sub;
}

constexpr int WTA_G = 4;  // pixels per 16-lane group (see wta_slab_kernel)

// What a launch of the slab WTA computes (one mode per launch, so that no load
// sits behind a runtime branch: the compiler then counts every load on every
// path and each wait covers only the loads it needs).
enum WtaMode : int {
    WM_RIGHT = 0,  // d* only (right views)
    WM_LEFT = 1,   // d*, sub-pixel disparity, valid := 1 (no right map)
    WM_LR = 2,     // ... and the LR check against wta_r
    WM_FEAT = 3,   // WM_LEFT and the network features (no right map)
    WM_FEAT_LR = 4 // WM_LR and the features
};

__host__ __device__ constexpr bool wm_lr(int m) { return m == WM_LR || m == WM_FEAT_LR; }
__host__ __device__ constexpr bool wm_feat(int m) { return m == WM_FEAT || m == WM_FEAT_LR; }

static int wta_mode(const WtaView &v)
{
    if (v.right_only) return WM_RIGHT;
    if (v.feat) return v.wta_r ? WM_FEAT_LR : WM_FEAT;
    return v.wta_r ? WM_LR : WM_LEFT;
}

// The slab WTA sums all eight direction slabs (a compile-time count, so no
// slab needs masking).
constexpr int WTA_NSLAB = 8;

// Result of one pixel's reduction, the same in every lane of its group.
struct WtaPx {
    int ds;                     // d*
    uint32_t smin, av, cv, s2;  // S(d*), S(d* - 1), S(d* + 1), min over |d - d*| >= 2
};

template <int K, int MODE>
__device__ __forceinline__ WtaPx wta_reduce(const WtaView &v, const u32x2 (&w)[2][8], int j)
{
    constexpr int D = 16 * K;
    uint32_t sv[2][4];
    int dd[2][8];
    slab_add<K>(w, j, WTA_NSLAB, sv, dd);
    uint32_t best = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 2; ++i)
        if (8 * (j + 16 * i) < D) {
#pragma unroll
            for (int e = 0; e < 8; ++e) best = min(best, (sv_val(sv, i, e) << 9) | (uint32_t)dd[i][e]);
        }
    const uint32_t key = row16_min(best);
    WtaPx r;
    r.ds = (int)(key & 511u);
    r.smin = key >> 9;
    r.av = r.cv = 0;
    r.s2 = 0xFFFFFFFFu;
    if constexpr (MODE != WM_RIGHT) neighbours<K, wm_feat(MODE)>(sv, dd, j, r.ds, r.av, r.cv, r.s2);
    return r;
}

// Stores of one pixel by the lanes of its group: d* (lane 0), and unless
// right-only the sub-pixel disparity, the LR check with the right map's value
// rq at x - d* and the valid flag (lane 0), and the four network features
// (lanes 4..7, one each; inten: the base image byte at the pixel).  The
// quotients of lane 0 and lanes 4..7 come from one FP32 division of the
// whole group, each lane with its own operands (the same operations as one
// lane doing them in turn).
template <int K, int MODE>
__device__ __forceinline__ void wta_finish(const WtaView &v, const WtaPx &r, int px, int x, int j, int rq,
                                           uint32_t inten)
{
    constexpr int D = 16 * K;
    if constexpr (MODE == WM_RIGHT) {
        if (j == 0) v.wta[px] = (int16_t)r.ds;
    } else {
        // Sub-pixel (lane 0): d* + (a - c) / (2 den) when 0 < d* < D - 1 and den > 0.
        const int den = (int)r.av - 2 * (int)r.smin + (int)r.cv;
        const bool para = r.ds > 0 && r.ds < D - 1 && den > 0;
        float num = (float)((int)r.av - (int)r.cv), dvs = (float)(2 * (den > 0 ? den : 1));
        if constexpr (wm_feat(MODE)) {
            const uint32_t s2 = r.s2 == 0xFFFFFFFFu ? r.smin : r.s2;
            const int f = j - 4;  // feature index of lanes 4..7
            if (f == 0) { num = (float)inten; dvs = 255.0f; }
            if (f == 1) { num = (float)r.ds; dvs = (float)(D > 1 ? D - 1 : 1); }
            if (f == 2) { num = (float)r.smin; dvs = (float)(8 * (SF_CMAX + v.P2)); }
            if (f == 3) { num = (float)s2; dvs = (float)(r.smin > 1 ? r.smin : 1u); }
        }
        const float q = num / dvs;
        if (j == 0) {
            const float sub = para ? (float)r.ds + q : (float)r.ds;
            int ok = 1;
            if constexpr (wm_lr(MODE)) {
                int diff = r.ds - rq;
                diff = diff < 0 ? -diff : diff;
                ok = (x - r.ds >= 0) && diff <= v.tol;
            }
            if (v.wta) v.wta[px] = (int16_t)r.ds;
            v.disp[px] = (ok || v.dense) ? sub : -1.0f;
            v.valid[px] = (uint8_t)ok;
        }
        if constexpr (wm_feat(MODE)) {
            const int f = j - 4;
            if (f >= 0 && f < 4) v.feat[(size_t)px * 4 + f] = (f == 1 && D <= 1) ? 0.0f : q;
        }
    }
}

// Each 16-lane group takes WTA_G pixels WTA_PPB apart, software-pipelined: the
// slabs (and image byte) of pixel g + 1 are loaded while pixel g is reduced,
// and pixel g's right-map value is loaded before pixel g - 1 is finished, so a
// wait for it never also waits for the next pixel's slabs (loads complete in
// issue order).  Past the end of the view the group re-reads its last pixel
// and stores nothing, so every load is issued on every path.  The pixel's row
// and column advance by WTA_PPB per step without a division.
template <int K, int MODE>
__global__ __launch_bounds__(WTA_NT) void wta_slab_kernel(WtaArgs a)
{
    int vi = 0;
    while ((int)blockIdx.x >= a.blk0[vi + 1]) ++vi;
    const WtaView v = a.v[vi];
    const int q = threadIdx.x >> 4, j = threadIdx.x & 15;
    const int px0 = ((int)blockIdx.x - a.blk0[vi]) * (WTA_PPB * WTA_G) + q;
    const int npx = v.H * v.W;
    constexpr int D = 16 * K;
    const size_t cells = (size_t)npx * D;
    if (px0 >= npx) return;  // uniform across the 16-lane group
    u32x2 w[2][2][8];
    uint32_t inten[2] = {0u, 0u};
    // (y, x) of pixel px0 + g WTA_PPB for the current step g, and of the next one.
    int cy = px0 / v.W, cx = px0 - cy * v.W;
    auto step_yx = [&](int &yy, int &xx) {
        xx += WTA_PPB;
        while (xx >= v.W) {
            xx -= v.W;
            ++yy;
        }
    };
    auto load_inten = [&](int yy, int xx) -> uint32_t {
        if (yy >= v.H) { yy = v.H - 1; xx = v.W - 1; }  // past the end: the last pixel
        return v.img[(size_t)yy * v.pitch + xx];
    };
    slab_load<K>(v.slab, cells, px0, j, WTA_NSLAB, w[0]);
    if constexpr (wm_feat(MODE)) inten[0] = load_inten(cy, cx);
    WtaPx prev{};
    int prev_px = 0, prev_x = 0, prev_rq = 0;
    uint32_t prev_in = 0u;  // inten of the previous pixel (its slot is reused by the prefetch)
#pragma unroll
    for (int g = 0; g < WTA_G; ++g) {
        const int px = min(px0 + g * WTA_PPB, npx - 1);
        int ny = cy, nx = cx;
        step_yx(ny, nx);
        if (g + 1 < WTA_G) {
            const int pn = min(px0 + (g + 1) * WTA_PPB, npx - 1);
            slab_load<K>(v.slab, cells, pn, j, WTA_NSLAB, w[(g + 1) & 1]);
            if constexpr (wm_feat(MODE)) inten[(g + 1) & 1] = load_inten(ny, nx);
            // Keep these loads ahead of pixel g's reduction (the scheduler would
            // otherwise sink them below its waits).
            __builtin_amdgcn_sched_barrier(0);
        }
        const WtaPx r = wta_reduce<K, MODE>(v, w[g & 1], j);
        const bool live = px0 + g * WTA_PPB < npx;
        const int y = live ? cy : v.H - 1, x = live ? cx : v.W - 1;
        int rq = 0;
        if constexpr (wm_lr(MODE)) {
            SF_BOUNDS(x - r.ds < v.W && y < v.H && y >= 0, CHK_WTA_LR);
            rq = v.wta_r[(size_t)y * v.W + max(x - r.ds, 0)];
        }
        if (g > 0 && px0 + (g - 1) * WTA_PPB < npx)
            wta_finish<K, MODE>(v, prev, prev_px, prev_x, j, prev_rq, prev_in);
        prev = r;
        prev_px = px;
        prev_x = x;
        prev_rq = rq;
        prev_in = inten[g & 1];
        cy = ny;
        cx = nx;
    }
    if (px0 + (WTA_G - 1) * WTA_PPB < npx)
        wta_finish<K, MODE>(v, prev, prev_px, prev_x, j, prev_rq, prev_in);
}

// Left WTA and the right map by diagonal search in one pass over the left
// slabs (a variant of the cited SGM method: the right view's disparity at q is
// the d minimising S_L(q + d, d), smallest d on ties, over q + d <= W - 1).
// One block per image row: each 16-lane group sums the slabs of one pixel x,
// takes its left WTA, and offers the key S_L(x, d) * 512 + d to the right
// pixel q = x - d with an LDS atomic minimum.  Once the whole row has been
// offered, the LR check reads the finished right map from LDS.
constexpr int DIAG_NT = 512;
constexpr int DIAG_MAXW = 4096;

template <int K>
__global__ __launch_bounds__(DIAG_NT) void wta_diag_slab_kernel(WtaArgs a)
{
    extern __shared__ uint32_t dg_lds[];
    int vi = 0;
    while ((int)blockIdx.x >= a.blk0[vi + 1]) ++vi;
    const WtaView v = a.v[vi];
    const int y = (int)blockIdx.x - a.blk0[vi];
    const int W = v.W;
    constexpr int D = 16 * K;
    uint32_t *bestr = dg_lds;                                  // [W] right-map keys
    float *dsl = reinterpret_cast<float *>(dg_lds + W);        // [W] left sub-pixel disparity
    int16_t *dl = reinterpret_cast<int16_t *>(dg_lds + 2 * W);  // [W] left d*
    for (int i = threadIdx.x; i < W; i += DIAG_NT) bestr[i] = 0xFFFFFFFFu;
    __syncthreads();
    const int g = threadIdx.x >> 4, j = threadIdx.x & 15;
    const size_t cells = (size_t)v.H * W * D;
    for (int x = g; x < W; x += DIAG_NT / 16) {
        uint32_t sv[2][4];
        int dd[2][8];
        slab_sums<K>(v.slab, cells, y * W + x, j, v.nslab, sv, dd);
        uint32_t best = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < 2; ++i)
            if (8 * (j + 16 * i) < D) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t k = (sv_val(sv, i, e) << 9) | (uint32_t)dd[i][e];
                    best = min(best, k);
                    const int q = x - dd[i][e];
                    if (q >= 0) atomicMin(&bestr[q], k);
                }
            }
        const uint32_t key = row16_min(best);
        const int ds = (int)(key & 511u);
        uint32_t av, cv, s2;
        neighbours<K, false>(sv, dd, j, ds, av, cv, s2);
        if (j == 0) {
            dl[x] = (int16_t)ds;
            dsl[x] = subpixel(ds, D, av, key >> 9, cv);
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < W; x += DIAG_NT) {
        const int ds = dl[x];
        const int qx = x - ds;
        int ok = 0;
        if (qx >= 0) {
            int diff = ds - (int)(bestr[qx] & 511u);
            diff = diff < 0 ? -diff : diff;
            ok = diff <= v.tol;
        }
        const size_t px = (size_t)y * W + x;
        if (v.wta) v.wta[px] = (int16_t)ds;
        if (v.wta_r_out) v.wta_r_out[px] = (int16_t)(bestr[x] & 511u);
        v.disp[px] = (ok || v.dense) ? dsl[x] : -1.0f;
        v.valid[px] = (uint8_t)ok;
    }
}

template <int K>
static void launch_wta_slab_mode(int mode, unsigned nblk, const WtaArgs &a, hipStream_t st)
{
    switch (mode) {
    case WM_RIGHT: hipLaunchKernelGGL((wta_slab_kernel<K, WM_RIGHT>), dim3(nblk), dim3(WTA_NT), 0, st, a); break;
    case WM_LEFT: hipLaunchKernelGGL((wta_slab_kernel<K, WM_LEFT>), dim3(nblk), dim3(WTA_NT), 0, st, a); break;
    case WM_LR: hipLaunchKernelGGL((wta_slab_kernel<K, WM_LR>), dim3(nblk), dim3(WTA_NT), 0, st, a); break;
    case WM_FEAT: hipLaunchKernelGGL((wta_slab_kernel<K, WM_FEAT>), dim3(nblk), dim3(WTA_NT), 0, st, a); break;
    default: hipLaunchKernelGGL((wta_slab_kernel<K, WM_FEAT_LR>), dim3(nblk), dim3(WTA_NT), 0, st, a); break;
    }
}

// One launch per run of consecutive views with the same mode (in practice all
// views of a call share it); the block offsets of each launch are computed
// here (a.blk0 is not read).
int launch_wta_slabs(const WtaArgs &a, hipStream_t st)
{
    for (int i = 0; i < a.n; ++i) {
        if (a.v[i].D != a.v[0].D) return fail(SF_EINVAL, "launch_wta_slabs: views of one launch need one D");
        if (a.v[i].nslab != WTA_NSLAB) return fail(SF_EINVAL, "launch_wta_slabs: the slab WTA sums all 8 slabs");
        if (a.v[i].feat && !a.v[i].img) return fail(SF_EINVAL, "launch_wta_slabs: features need the base image");
    }
    const int K = a.v[0].D / 16;
    if (K != 2 && K != 4 && K != 6 && K != 8 && K != 10 && K != 12 && K != 14 && K != 16)
        return fail(SF_EUNSUPPORTED, "launch_wta_slabs: unsupported D");
    for (int i0 = 0; i0 < a.n;) {
        const int mode = wta_mode(a.v[i0]);
        int i1 = i0 + 1;
        while (i1 < a.n && wta_mode(a.v[i1]) == mode) ++i1;
        WtaArgs g{};
        long long tot = 0;
        for (int i = i0; i < i1; ++i) {
            g.v[i - i0] = a.v[i];
            g.blk0[i - i0] = (int)tot;
            tot += ((long long)a.v[i].H * a.v[i].W + WTA_PPB * WTA_G - 1) / (WTA_PPB * WTA_G);
        }
        g.n = i1 - i0;
        for (int i = g.n; i <= STAGE_MAXV; ++i) g.blk0[i] = (int)tot;
        if (tot > 0x7FFFFFFFLL) return fail(SF_EINVAL, "launch_wta_slabs: grid too large");
        if (tot > 0) {
            ProfScope prof(mode == WM_RIGHT ? "wta_slab_right" : "wta_slab_left", st);
            switch (K) {
            case 2: launch_wta_slab_mode<2>(mode, (unsigned)tot, g, st); break;
            case 4: launch_wta_slab_mode<4>(mode, (unsigned)tot, g, st); break;
            case 6: launch_wta_slab_mode<6>(mode, (unsigned)tot, g, st); break;
            case 8: launch_wta_slab_mode<8>(mode, (unsigned)tot, g, st); break;
            case 10: launch_wta_slab_mode<10>(mode, (unsigned)tot, g, st); break;
            case 12: launch_wta_slab_mode<12>(mode, (unsigned)tot, g, st); break;
            case 14: launch_wta_slab_mode<14>(mode, (unsigned)tot, g, st); break;
            default: launch_wta_slab_mode<16>(mode, (unsigned)tot, g, st); break;
            }
            const int rc = launch_status("wta_slab_kernel");
            if (rc) return rc;
        }
        i0 = i1;
    }
    return SF_OK;
}

int launch_wta_diag_slabs(WtaArgs &a, hipStream_t st)
{
    long long tot = 0;
    for (int i = 0; i < a.n; ++i) {
        a.blk0[i] = (int)tot;
        tot += a.v[i].H;
    }
    for (int i = a.n; i <= STAGE_MAXV; ++i) a.blk0[i] = (int)tot;
    if (tot <= 0) return SF_OK;
    int maxw = 0;
    for (int i = 0; i < a.n; ++i) {
        if (a.v[i].D != a.v[0].D) return fail(SF_EINVAL, "launch_wta_diag_slabs: views of one launch need one D");
        if (a.v[i].nslab < 1 || a.v[i].nslab > 8) return fail(SF_EINVAL, "launch_wta_diag_slabs: nslab must be in [1, 8]");
        if (a.v[i].W > DIAG_MAXW) return fail(SF_EUNSUPPORTED, "launch_wta_diag_slabs: W > 4096");
        maxw = max(maxw, a.v[i].W);
    }
    const size_t lds = (size_t)maxw * (4 + 4 + 2);
    ProfScope prof("wta_diag", st);
    switch (a.v[0].D / 16) {
#define SF_DIAG_CASE(KK)                                                                            \
    case KK:                                                                                        \
        hipLaunchKernelGGL(wta_diag_slab_kernel<KK>, dim3((unsigned)tot), dim3(DIAG_NT), lds, st, a); \
        break;
        SF_DIAG_CASE(2) SF_DIAG_CASE(4) SF_DIAG_CASE(6) SF_DIAG_CASE(8) SF_DIAG_CASE(10)
        SF_DIAG_CASE(12) SF_DIAG_CASE(14) SF_DIAG_CASE(16)
#undef SF_DIAG_CASE
    default: return fail(SF_EUNSUPPORTED, "launch_wta_diag_slabs: unsupported D");
    }
    return launch_status("wta_diag_slab_kernel");
}

// d*_R by the diagonal search on a u16 volume S_L (the stage entry point).
// One 16-lane group per right pixel q; lane j scans d = j, j + 16, ...
__global__ __launch_bounds__(WTA_NT) void wta_diag_right_kernel(const uint16_t *__restrict__ S,
                                                               int H, int W, int D,
                                                               int16_t *__restrict__ wta_r)
{
    const int px = blockIdx.x * WTA_PPB + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    if (px >= H * W) return;
    const int y = px / W, q = px - y * W;
    uint32_t best = 0xFFFFFFFFu;
    for (int d = j; d < D && q + d < W; d += 16)
        best = min(best, ((uint32_t)S[((size_t)y * W + q + d) * D + d] << 9) | (uint32_t)d);
    best = row16_min(best);
    if (j == 0) wta_r[px] = (int16_t)(best & 511u);
}

// LR mask: valid iff x - d*_L >= 0 and |d*_L - d*_R(x - d*_L)| <= tol;
// disp = dsub where valid, else -1.
__global__ __launch_bounds__(256) void lr_check_kernel(const int16_t *__restrict__ wl,
                                                       const int16_t *__restrict__ wr,
                                                       const float *__restrict__ dsub, int H, int W,
                                                       int tol, uint8_t *__restrict__ valid,
                                                       float *__restrict__ disp)
{
    const int px = blockIdx.x * 256 + threadIdx.x;
    if (px >= H * W) return;
    const int y = px / W, x = px - y * W;
    const int dl = wl[px], q = x - dl;
    int ok = 0;
    if (q >= 0) {
        SF_BOUNDS(q < W, CHK_WTA_LR);
        int diff = dl - (int)wr[(size_t)y * W + q];
        diff = diff < 0 ? -diff : diff;
        ok = diff <= tol;
    }
    valid[px] = (uint8_t)ok;
    disp[px] = ok ? dsub[px] : -1.0f;
}

// 3x3 median with clamp-to-edge; with a mask, pixels outside it get -1.  The
// 16x16 tile plus a one-pixel halo is staged in LDS; the median of nine is a
// fixed network of 19 compare-exchanges (min/max return one of their inputs,
// so the result is one of the nine values bit for bit).
constexpr int MED_T = 16;

__device__ __forceinline__ void cx(float &a, float &b)
{
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    a = lo;
    b = hi;
}

__global__ __launch_bounds__(MED_T *MED_T) void median3x3_kernel(const float *__restrict__ in,
                                                                 const uint8_t *__restrict__ mask,
                                                                 int H, int W,
                                                                 float *__restrict__ out)
{
    __shared__ float t[MED_T + 2][MED_T + 2];
    const int x0 = blockIdx.x * MED_T, y0 = blockIdx.y * MED_T;
    const int tid = threadIdx.y * MED_T + threadIdx.x;
    for (int i = tid; i < (MED_T + 2) * (MED_T + 2); i += MED_T * MED_T) {
        const int ly = i / (MED_T + 2), lx = i - ly * (MED_T + 2);
        const int gy = min(max(y0 + ly - 1, 0), H - 1), gx = min(max(x0 + lx - 1, 0), W - 1);
        t[ly][lx] = in[(size_t)gy * W + gx];
    }
    __syncthreads();
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    if (x >= W || y >= H) return;
    float p[9];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) p[3 * j + i] = t[threadIdx.y + j][threadIdx.x + i];
    cx(p[1], p[2]); cx(p[4], p[5]); cx(p[7], p[8]);
    cx(p[0], p[1]); cx(p[3], p[4]); cx(p[6], p[7]);
    cx(p[1], p[2]); cx(p[4], p[5]); cx(p[7], p[8]);
    cx(p[0], p[3]); cx(p[5], p[8]); cx(p[4], p[7]);
    cx(p[3], p[6]); cx(p[1], p[4]); cx(p[2], p[5]);
    cx(p[4], p[7]); cx(p[4], p[2]); cx(p[6], p[4]);
    cx(p[4], p[2]);
    const size_t px = (size_t)y * W + x;
    out[px] = (!mask || mask[px]) ? p[4] : -1.0f;
}

int launch_median_mask(const float *dense, const uint8_t *mask, int H, int W, float *out,
                       hipStream_t st)
{
    dim3 grid((W + MED_T - 1) / MED_T, (H + MED_T - 1) / MED_T);
    ProfScope prof("median3x3", st);
    hipLaunchKernelGGL(median3x3_kernel, grid, dim3(MED_T, MED_T), 0, st, dense, mask, H, W, out);
    return launch_status("median3x3_kernel");
}

}  // namespace sf

using namespace sf;

extern "C" int sf_wta_lr(const uint16_t *S_left, const uint16_t *S_right, const uint8_t *img_left,
                         int pitch, int H, int W, int D, int P2, int lr_tol, int16_t *wta_left,
                         int16_t *wta_right, float *disp, uint8_t *valid, float *feat, void *stream)
{
    clear_error();
    SF_REQUIRE(S_left && wta_left && disp && valid, SF_EINVAL, "sf_wta_lr: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_wta_lr: H and W must be positive");
    SF_REQUIRE((long long)H * W <= (1LL << 30), SF_EINVAL, "sf_wta_lr: image too large");
    SF_REQUIRE(D >= 1 && D <= SF_DMAX, SF_EINVAL, "sf_wta_lr: D must be in [1, 256]");
    SF_REQUIRE(lr_tol >= 0, SF_EINVAL, "sf_wta_lr: lr_tol < 0");
    SF_REQUIRE(!S_right || wta_right, SF_EINVAL, "sf_wta_lr: S_right needs wta_right");
    SF_REQUIRE(!feat || (img_left && pitch >= W), SF_EINVAL,
               "sf_wta_lr: features need img_left with pitch >= W");
    SF_REQUIRE(P2 >= 0 && P2 <= 8000, SF_EINVAL, "sf_wta_lr: P2 out of range");
    hipStream_t st = as_stream(stream);
    const int npx = H * W;
    const int nblk = (npx + WTA_PPB - 1) / WTA_PPB;
    if (S_right) {
        ProfScope prof("wta_right", as_stream(stream));
        hipLaunchKernelGGL(wta_right_kernel, dim3(nblk), dim3(WTA_NT), 0, st, S_right, npx, D,
                           wta_right);
        int rc = launch_status("wta_right_kernel");
        if (rc) return rc;
    }
    ProfScope prof("wta_left", as_stream(stream));
    hipLaunchKernelGGL(wta_left_kernel, dim3(nblk), dim3(WTA_NT), 0, st, S_left,
                       S_right ? wta_right : nullptr, img_left, pitch, H, W, D, P2, lr_tol,
                       wta_left, disp, valid, feat);
    return launch_status("wta_left_kernel");
}

extern "C" int sf_wta_right_diag(const uint16_t *S_left, int H, int W, int D, int16_t *wta_right,
                                 void *stream)
{
    clear_error();
    SF_REQUIRE(S_left && wta_right, SF_EINVAL, "sf_wta_right_diag: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_wta_right_diag: H and W must be positive");
    SF_REQUIRE((long long)H * W <= (1LL << 30), SF_EINVAL, "sf_wta_right_diag: image too large");
    SF_REQUIRE(D >= 1 && D <= SF_DMAX, SF_EINVAL, "sf_wta_right_diag: D must be in [1, 256]");
    const int npx = H * W;
    ProfScope prof("wta_right_diag", as_stream(stream));
    hipLaunchKernelGGL(wta_diag_right_kernel, dim3((npx + WTA_PPB - 1) / WTA_PPB), dim3(WTA_NT), 0,
                       as_stream(stream), S_left, H, W, D, wta_right);
    return launch_status("wta_diag_right_kernel");
}

extern "C" int sf_lr_check(const int16_t *wta_left, const int16_t *wta_right, const float *dsub,
                           int H, int W, int lr_tol, uint8_t *valid, float *disp, void *stream)
{
    clear_error();
    SF_REQUIRE(wta_left && wta_right && dsub && valid && disp, SF_EINVAL, "sf_lr_check: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_lr_check: H and W must be positive");
    SF_REQUIRE((long long)H * W <= (1LL << 30), SF_EINVAL, "sf_lr_check: image too large");
    SF_REQUIRE(lr_tol >= 0, SF_EINVAL, "sf_lr_check: lr_tol < 0");
    const int npx = H * W;
    hipLaunchKernelGGL(lr_check_kernel, dim3((npx + 255) / 256), dim3(256), 0, as_stream(stream),
                       wta_left, wta_right, dsub, H, W, lr_tol, valid, disp);
    return launch_status("lr_check_kernel");
}

extern "C" int sf_median3x3(const float *in, const uint8_t *mask, int H, int W, float *out,
                            void *stream)
{
    clear_error();
    SF_REQUIRE(in && out, SF_EINVAL, "sf_median3x3: NULL pointer");
    SF_REQUIRE(in != out, SF_EINVAL, "sf_median3x3: in and out must not be the same buffer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_median3x3: H and W must be positive");
    SF_REQUIRE(H <= 65535 * 16, SF_EINVAL, "sf_median3x3: H too large");
    return launch_median_mask(in, mask, H, W, out, as_stream(stream));
}
