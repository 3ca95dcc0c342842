// Winner-take-all with parabolic sub-pixel refinement, the left-right
// consistency check (paper Sec. 3.1: two computed disparity maps are compared
// and inconsistent pixels removed, leaving a non-dense map) and the per-pixel
// features of the learned stand-in for that check.
//
// One 16-lane DPP row per pixel: lane j reads disparities [4c, 4c+4) for
// c = j, j+16, ... (128 contiguous bytes per row per load), the (S, d) minimum
// is a row butterfly on the key S * 512 + d, so ties go to the smallest d.
#include "sf_internal.hpp"
#include "stages.hpp"

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

template <int K>
__global__ __launch_bounds__(WTA_NT) void wta_slab_kernel(WtaArgs a)
{
    int vi = 0;
    while ((int)blockIdx.x >= a.blk0[vi + 1]) ++vi;
    const WtaView v = a.v[vi];
    const int q = threadIdx.x >> 4, j = threadIdx.x & 15;
    const int px = ((int)blockIdx.x - a.blk0[vi]) * WTA_PPB + q;
    const int npx = v.H * v.W;
    if (px >= npx) return;
    constexpr int D = 16 * K;
    const size_t cells = (size_t)npx * D;
    uint32_t sv[2][4];
    int dd[2][8];
    uint32_t best = 0xFFFFFFFFu;
    // All slab loads of the lane are issued before any is used (slabs past
    // nslab re-read the last one and are masked to zero), so each wave keeps
    // up to 16 loads in flight.
    const int ns = v.nslab;
    u32x2 w[2][8];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = j + 16 * i;
        if (8 * c < D) {
            const uint8_t *src = v.slab + (size_t)px * D + 8 * c;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                w[i][k] = __builtin_nontemporal_load(
                    reinterpret_cast<const u32x2 *>(src + (size_t)min(k, ns - 1) * cells));
        }
    }
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
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t val = (e & 1) ? (sv[i][e >> 1] >> 16) : (sv[i][e >> 1] & 0xFFFFu);
                best = min(best, (val << 9) | (uint32_t)dd[i][e]);
            }
        }
    }
    const uint32_t key = row16_min(best);
    const int ds = (int)(key & 511u);
    const uint32_t smin = key >> 9;
    if (v.right_only) {
        if (j == 0) v.wta[px] = (int16_t)ds;
        return;
    }
    uint32_t av = 0, cv = 0, s2 = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = j + 16 * i;
        if (8 * c < D) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int d = dd[i][e];
                const uint32_t val = (e & 1) ? (sv[i][e >> 1] >> 16) : (sv[i][e >> 1] & 0xFFFFu);
                if (d == ds - 1) av = val;
                if (d == ds + 1) cv = val;
                const int gap = d > ds ? d - ds : ds - d;
                if (gap >= 2) s2 = min(s2, val);
            }
        }
    }
    av = row16_max(av);
    cv = row16_max(cv);
    s2 = row16_min(s2);
    if (j != 0) return;
    const int y = px / v.W, x = px - y * v.W;
    float sub = (float)ds;
    if (ds > 0 && ds < D - 1) {
        const int den = (int)av - 2 * (int)smin + (int)cv;
        if (den > 0) sub = (float)ds + (float)((int)av - (int)cv) / (float)(2 * den);
    }
    int ok = 1;
    if (v.wta_r) {
        const int qx = x - ds;
        ok = 0;
        if (qx >= 0) {
            int diff = ds - (int)v.wta_r[(size_t)y * v.W + qx];
            diff = diff < 0 ? -diff : diff;
            ok = diff <= v.tol;
        }
    }
    if (v.wta) v.wta[px] = (int16_t)ds;
    v.disp[px] = ok ? sub : -1.0f;
    v.valid[px] = (uint8_t)ok;
    if (v.feat) {
        if (s2 == 0xFFFFFFFFu) s2 = smin;
        float4 f;
        f.x = (float)v.img[(size_t)y * v.pitch + x] / 255.0f;
        f.y = D > 1 ? (float)ds / (float)(D - 1) : 0.0f;
        f.z = (float)smin / (float)(8 * (SF_CMAX + v.P2));
        f.w = (float)s2 / (float)(smin > 1 ? smin : 1u);
        reinterpret_cast<float4 *>(v.feat)[px] = f;
    }
}

int launch_wta_slabs(WtaArgs &a, hipStream_t st)
{
    long long tot = 0;
    for (int i = 0; i < a.n; ++i) {
        a.blk0[i] = (int)tot;
        tot += ((long long)a.v[i].H * a.v[i].W + WTA_PPB - 1) / WTA_PPB;
    }
    for (int i = a.n; i <= STAGE_MAXV; ++i) a.blk0[i] = (int)tot;
    if (tot <= 0) return SF_OK;
    if (tot > 0x7FFFFFFFLL) return fail(SF_EINVAL, "launch_wta_slabs: grid too large");
    for (int i = 0; i < a.n; ++i) {
        if (a.v[i].D != a.v[0].D) return fail(SF_EINVAL, "launch_wta_slabs: views of one launch need one D");
        if (a.v[i].nslab < 1 || a.v[i].nslab > 8) return fail(SF_EINVAL, "launch_wta_slabs: nslab must be in [1, 8]");
    }
    ProfScope prof(a.v[0].right_only ? "wta_slab_right" : "wta_slab_left", st);
    switch (a.v[0].D / 16) {
#define SF_WTA_CASE(KK)                                                                             \
    case KK:                                                                                        \
        hipLaunchKernelGGL(wta_slab_kernel<KK>, dim3((unsigned)tot), dim3(WTA_NT), 0, st, a);        \
        break;
        SF_WTA_CASE(2) SF_WTA_CASE(4) SF_WTA_CASE(6) SF_WTA_CASE(8) SF_WTA_CASE(10) SF_WTA_CASE(12)
        SF_WTA_CASE(14) SF_WTA_CASE(16)
#undef SF_WTA_CASE
    default: return fail(SF_EUNSUPPORTED, "launch_wta_slabs: unsupported D");
    }
    return launch_status("wta_slab_kernel");
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
