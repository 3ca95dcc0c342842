// Optical-flow stand-in for the flow input of the scene-flow combination.  The
// paper takes its flow from Flow Fields+ (Sec. 3.2): matches found on a coarse
// level, propagated to neighbours and refined by random search under a patch
// data term, lifted level by level to full resolution and filtered by
// consistency with the inverse flow.  This module follows that outline with
// choices of its own:
//   * pyramid: 2x2 box means (a+b+c+d+2)/4, odd borders clamped;
//   * data term: the 9x7 census of the stereo path at every level; the cost of
//     integer flow f at x is the sum of the Hamming distances of the census at
//     x + o and x + f + o over o in {-2, 0, 2}^2 (coordinates clamped), and a
//     flow whose target leaves the image is no candidate;
//   * each iteration updates all pixels from the previous field: own f, the f
//     of the neighbours at distance 1 then 4 (left, right, up, down), then
//     random search around the best so far with radii R_l >> k (R_l = max(1,
//     R >> l), capped at fine_radius below the coarsest level when
//     fine_radius > 0), offsets drawn
//     from SplitMix64 (counter = (((level*64 + iter)*64 + k)*65536 + y/8)*65536
//     + x/8: one offset per 8x8 tile, so a wave's candidate loads stay mostly
//     contiguous); the first candidate with the lowest cost wins;
//   * coarse to fine: f = 0 on the coarsest level, f = 2 f(x/2, y/2) with the
//     target clamped into the image when moving one level finer;
//   * forward-backward check: F(x) is kept iff |F(x) + B(x + F(x))| <= tol in
//     both components (B from the second image to the first, seed ^ 0x5bd1e995).
// All integer: results are reproducible bit for bit.  One thread per pixel,
// 16x16 blocks; the census words of both images come through L1/L2.
#include "sf_check.hpp"
#include "sf_internal.hpp"
#include "stages.hpp"

SF_CHECK_TU(flow)

namespace sf {

constexpr int FL_T = 16;
constexpr int FL_MAXLEV = 16;

// Two images per launch (blockIdx.y selects the image).
struct PyrArgs {
    const uint8_t *in[2];
    uint8_t *out[2];
};

__global__ __launch_bounds__(256) void pyr_down_kernel(PyrArgs a, int H, int W, int pitch)
{
    const uint8_t *__restrict__ in = a.in[blockIdx.y];
    uint8_t *__restrict__ out = a.out[blockIdx.y];
    const int w = (W + 1) / 2, h = (H + 1) / 2;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= w * h) return;
    const int y = i / w, x = i - y * w;
    const int x0 = 2 * x, y0 = 2 * y;
    const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
    const int s = in[(size_t)y0 * pitch + x0] + in[(size_t)y0 * pitch + x1] +
                  in[(size_t)y1 * pitch + x0] + in[(size_t)y1 * pitch + x1];
    out[i] = (uint8_t)((s + 2) >> 2);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Cost of flow (fu, fv) at (x, y) given the pixel's own nine census words a[]:
// -1 when the target leaves the image.
__device__ __forceinline__ int flow_cost(const uint64_t (&a)[9], const uint64_t *__restrict__ c1,
                                         int H, int W, int x, int y, int fu, int fv)
{
    const int tx = x + fu, ty = y + fv;
    if (tx < 0 || tx > W - 1 || ty < 0 || ty > H - 1) return -1;
    int s = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const size_t row = (size_t)min(max(ty + 2 * j - 2, 0), H - 1) * W;
        SF_BOUNDS(row < (size_t)H * W && tx >= 0 && tx < W, CHK_FLOW_SAMPLE);
#pragma unroll
        for (int i = 0; i < 3; ++i) s += __popcll(a[3 * j + i] ^ c1[row + min(max(tx + 2 * i - 2, 0), W - 1)]);
    }
    return s;
}

// One iteration of both flow directions (blockIdx.z = direction d: the flow
// from image d to image 1 - d, with its own seed and flow buffers).
struct PmArgs {
    const uint64_t *c0[2], *c1[2];  // census of the source and target image
    const short2 *fin[2];
    short2 *fout[2];
    uint64_t seed[2];
};

__global__ __launch_bounds__(FL_T *FL_T) void pm_iter_kernel(PmArgs pa, int H, int W, int level,
                                                             int iter, int Rl)
{
    const int dz = blockIdx.z;
    const uint64_t *__restrict__ c0 = pa.c0[dz];
    const uint64_t *__restrict__ c1 = pa.c1[dz];
    const short2 *__restrict__ fin = pa.fin[dz];
    short2 *__restrict__ fout = pa.fout[dz];
    const uint64_t seed = pa.seed[dz];
    const int x = blockIdx.x * FL_T + threadIdx.x, y = blockIdx.y * FL_T + threadIdx.y;
    if (x >= W || y >= H) return;
    uint64_t a[9];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const size_t row = (size_t)min(max(y + 2 * j - 2, 0), H - 1) * W;
#pragma unroll
        for (int i = 0; i < 3; ++i) a[3 * j + i] = c0[row + min(max(x + 2 * i - 2, 0), W - 1)];
    }
    const size_t idx = (size_t)y * W + x;
    const short2 f0 = fin[idx];
    int bu = f0.x, bv = f0.y;
    int best = flow_cost(a, c1, H, W, x, y, bu, bv);
    if (best < 0) best = 1 << 30;
    // Propagation: distance 1 then 4; left, right, up, down.
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int d = s == 0 ? 1 : 4;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int nx = x + (n == 0 ? -d : (n == 1 ? d : 0));
            const int ny = y + (n == 2 ? -d : (n == 3 ? d : 0));
            if (nx < 0 || nx > W - 1 || ny < 0 || ny > H - 1) continue;
            const short2 c = fin[(size_t)ny * W + nx];
            // A candidate equal to the best so far has its cost and cannot win
            // (only a strictly lower cost replaces): skip its evaluation.
            if (c.x == bu && c.y == bv) continue;
            const int cc = flow_cost(a, c1, H, W, x, y, c.x, c.y);
            if (cc >= 0 && cc < best) {
                best = cc;
                bu = c.x;
                bv = c.y;
            }
        }
    }
    // Random search around the best so far, radii halving from Rl.
    for (int k = 0; (Rl >> k) >= 1; ++k) {
        const int r = Rl >> k;
        const uint64_t ctr =
            ((((uint64_t)level * 64 + (uint64_t)iter) * 64 + (uint64_t)k) * 65536 + (uint64_t)(y >> 3)) *
                65536 +
            (uint64_t)(x >> 3);
        const uint64_t h = splitmix64(seed, ctr);
        const uint32_t m = (uint32_t)(2 * r + 1);
        const int ou = (int)((uint32_t)(h & 0xFFFFu) % m) - r;
        const int ov = (int)((uint32_t)((h >> 16) & 0xFFFFu) % m) - r;
        if (ou == 0 && ov == 0) continue;  // the best itself: cannot win
        const int cu = bu + ou, cv = bv + ov;
        const int cc = flow_cost(a, c1, H, W, x, y, cu, cv);
        if (cc >= 0 && cc < best) {
            best = cc;
            bu = cu;
            bv = cv;
        }
    }
    fout[idx] = make_short2((short)bu, (short)bv);
}

// Start of a level: zero on the coarsest, else twice the coarser flow at
// (x/2, y/2) with the target clamped into the image.
// Both directions per launch (blockIdx.y = direction).
struct InitArgs {
    const short2 *coarse[2];  // NULL on the coarsest level
    short2 *out[2];
};

__global__ __launch_bounds__(256) void flow_init_kernel(InitArgs a, int hc, int wc, int H, int W)
{
    const short2 *__restrict__ coarse = a.coarse[blockIdx.y];
    short2 *__restrict__ out = a.out[blockIdx.y];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= H * W) return;
    const int y = i / W, x = i - y * W;
    if (!coarse) {
        out[i] = make_short2(0, 0);
        return;
    }
    const short2 c = coarse[(size_t)min(y / 2, hc - 1) * wc + min(x / 2, wc - 1)];
    const int fu = 2 * c.x, fv = 2 * c.y;
    out[i] = make_short2((short)(min(max(x + fu, 0), W - 1) - x), (short)(min(max(y + fv, 0), H - 1) - y));
}

__global__ __launch_bounds__(256) void fb_check_kernel(const short2 *__restrict__ F,
                                                       const short2 *__restrict__ B, int H, int W,
                                                       int tol, float2 *__restrict__ out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= H * W) return;
    const int y = i / W, x = i - y * W;
    const short2 f = F[i];
    const int tx = x + f.x, ty = y + f.y;
    bool ok = false;
    if (tx >= 0 && tx < W && ty >= 0 && ty < H) {
        const short2 b = B[(size_t)ty * W + tx];
        const int eu = f.x + b.x, ev = f.y + b.y;
        ok = eu >= -tol && eu <= tol && ev >= -tol && ev <= tol;
    }
    const float nanv = __builtin_nanf("");
    out[i] = ok ? make_float2((float)f.x, (float)f.y) : make_float2(nanv, nanv);
}

struct FlowLayout {
    int levels;
    int h[FL_MAXLEV], w[FL_MAXLEV];
    size_t off_img[2][FL_MAXLEV];  // level >= 1 images of A and B
    size_t off_cen[2][FL_MAXLEV];  // census of A and B per level
    size_t off_f[2][2];            // ping-pong flow buffers per direction (full size)
    size_t bytes;
};

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

static FlowLayout flow_layout(int H, int W, int levels)
{
    FlowLayout L{};
    L.levels = levels;
    L.h[0] = H;
    L.w[0] = W;
    for (int l = 1; l < levels; ++l) {
        L.h[l] = (L.h[l - 1] + 1) / 2;
        L.w[l] = (L.w[l - 1] + 1) / 2;
    }
    size_t off = 0;
    for (int s = 0; s < 2; ++s)
        for (int l = 0; l < levels; ++l) {
            const size_t n = (size_t)L.h[l] * L.w[l];
            if (l > 0) {
                L.off_img[s][l] = off;
                off += al256(n);
            }
            L.off_cen[s][l] = off;
            off += al256(n * 8);
        }
    for (int d = 0; d < 2; ++d)
        for (int k = 0; k < 2; ++k) {
            L.off_f[d][k] = off;
            off += al256((size_t)H * W * 4);
        }
    L.bytes = off;
    return L;
}

// Integer flows from image 0 to image 1 (F) and from image 1 to image 0 (B)
// over the prepared pyramid / census, both directions in every launch; the last
// iteration of the finest level writes F and B.
static int run_directions(const FlowLayout &L, uint8_t *ws, int iters, int R, int fine_radius,
                          const uint64_t seed[2], short2 *F, short2 *B, hipStream_t st)
{
    short2 *buf[2][2];
    for (int d = 0; d < 2; ++d)
        for (int k = 0; k < 2; ++k) buf[d][k] = reinterpret_cast<short2 *>(ws + L.off_f[d][k]);
    short2 *result[2] = {F, B};
    int cur = 0;  // both directions keep their current field in buf[d][cur]
    for (int l = L.levels - 1; l >= 0; --l) {
        const int h = L.h[l], w = L.w[l], n = h * w;
        const bool coarsest = l == L.levels - 1;
        const int dst = coarsest ? cur : 1 - cur;
        InitArgs ia{};
        for (int d = 0; d < 2; ++d) {
            ia.coarse[d] = coarsest ? nullptr : buf[d][cur];
            ia.out[d] = buf[d][dst];
        }
        hipLaunchKernelGGL(flow_init_kernel, dim3((n + 255) / 256, 2), dim3(256), 0, st, ia,
                           coarsest ? 1 : L.h[l + 1], coarsest ? 1 : L.w[l + 1], h, w);
        cur = dst;
        dim3 grid((w + FL_T - 1) / FL_T, (h + FL_T - 1) / FL_T, 2);
        int Rl = max(1, R >> l);
        if (l < L.levels - 1 && fine_radius > 0 && Rl > fine_radius) Rl = fine_radius;
        for (int it = 0; it < iters; ++it) {
            const bool last = l == 0 && it == iters - 1;
            PmArgs pa{};
            for (int d = 0; d < 2; ++d) {
                pa.c0[d] = reinterpret_cast<const uint64_t *>(ws + L.off_cen[d][l]);
                pa.c1[d] = reinterpret_cast<const uint64_t *>(ws + L.off_cen[1 - d][l]);
                pa.fin[d] = buf[d][cur];
                pa.fout[d] = last ? result[d] : buf[d][1 - cur];
                pa.seed[d] = seed[d];
            }
            hipLaunchKernelGGL(pm_iter_kernel, grid, dim3(FL_T, FL_T), 0, st, pa, h, w, l, it, Rl);
            cur = 1 - cur;
        }
    }
    return launch_status("pm_iter_kernel");
}

}  // namespace sf

using namespace sf;

extern "C" size_t sf_flow_workspace_bytes(int H, int W, int levels)
{
    if (H <= 0 || W <= 0 || levels < 1 || levels > FL_MAXLEV) return 0;
    return flow_layout(H, W, levels).bytes;
}

extern "C" int sf_flow(const uint8_t *L0, const uint8_t *L1, int pitch, int H, int W, int levels,
                       int iters, int R, int fine_radius, uint64_t seed, int tol, int16_t *F,
                       int16_t *B, float *flow, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(L0 && L1 && F && B && flow, SF_EINVAL, "sf_flow: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0 && H <= 16383 && W <= 16383, SF_EINVAL, "sf_flow: H and W must be in [1, 16383]");
    SF_REQUIRE(pitch >= W, SF_EINVAL, "sf_flow: pitch < W");
    SF_REQUIRE(levels >= 1 && levels <= FL_MAXLEV, SF_EINVAL, "sf_flow: levels must be in [1, 16]");
    SF_REQUIRE(iters >= 1 && iters <= 63, SF_EINVAL, "sf_flow: iters must be in [1, 63]");
    SF_REQUIRE(R >= 1 && R <= 16383, SF_EINVAL, "sf_flow: R must be in [1, 16383]");
    SF_REQUIRE(fine_radius >= 0, SF_EINVAL, "sf_flow: fine_radius < 0");
    SF_REQUIRE(tol >= 0, SF_EINVAL, "sf_flow: tol < 0");
    const FlowLayout L = flow_layout(H, W, levels);
    SF_REQUIRE(workspace, SF_EINVAL, "sf_flow: NULL workspace");
    SF_REQUIRE(ws_bytes >= L.bytes, SF_ENOMEM, "sf_flow: workspace too small");
    SF_REQUIRE((reinterpret_cast<uintptr_t>(F) | reinterpret_cast<uintptr_t>(B)) % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(flow) % 8 == 0,
               SF_EINVAL, "sf_flow: F, B need 4-byte and flow 8-byte alignment");
    hipStream_t st = as_stream(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    ProfScope prof("flow", st);
    // Pyramids of both images, then the census of every level (both images per launch).
    const uint8_t *src[2] = {L0, L1};
    for (int l = 1; l < levels; ++l) {
        PyrArgs pa{};
        for (int s = 0; s < 2; ++s) {
            pa.in[s] = l == 1 ? src[s] : ws + L.off_img[s][l - 1];
            pa.out[s] = ws + L.off_img[s][l];
        }
        const int n = L.h[l] * L.w[l];
        hipLaunchKernelGGL(pyr_down_kernel, dim3((n + 255) / 256, 2), dim3(256), 0, st, pa, L.h[l - 1],
                           L.w[l - 1], l == 1 ? pitch : L.w[l - 1]);
    }
    int rc = launch_status("pyr_down_kernel");
    if (rc) return rc;
    for (int l = 0; l < levels; ++l) {
        CensusArgs ca{};
        for (int s = 0; s < 2; ++s) {
            ca.img[s] = l == 0 ? src[s] : ws + L.off_img[s][l];
            ca.pitch[s] = l == 0 ? pitch : L.w[l];
            ca.out[s] = reinterpret_cast<uint64_t *>(ws + L.off_cen[s][l]);
        }
        ca.n = 2;
        ca.H = L.h[l];
        ca.W = L.w[l];
        if ((rc = launch_census(ca, st))) return rc;
    }
    const uint64_t seeds[2] = {seed, seed ^ 0x5bd1e995ULL};
    if ((rc = run_directions(L, ws, iters, R, fine_radius, seeds, reinterpret_cast<short2 *>(F),
                             reinterpret_cast<short2 *>(B), st)))
        return rc;
    const int n = H * W;
    hipLaunchKernelGGL(fb_check_kernel, dim3((n + 255) / 256), dim3(256), 0, st,
                       reinterpret_cast<const short2 *>(F), reinterpret_cast<const short2 *>(B), H, W, tol,
                       reinterpret_cast<float2 *>(flow));
    return launch_status("fb_check_kernel");
}
