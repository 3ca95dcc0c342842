// Census transform and Hamming matching-cost volume (the matching cost inside
// SGM, paper Sec. 3.1; the 9x7 census and Hamming distance are the workload's
// choice, the paper names no cost).
#include "sf_internal.hpp"
#include "stages.hpp"

namespace sf {

constexpr int CEN_TW = 64;  // tile width  (one wave per tile row)
constexpr int CEN_TH = 4;   // tile height (four waves)
constexpr int CEN_RX = 4;   // window half-width  (9 wide)
constexpr int CEN_RY = 3;   // window half-height (7 tall)

// One thread per pixel; the (TH + 6) x (TW + 8) window of the tile is staged
// in LDS with clamp-to-edge, coalesced along rows.
__global__ __launch_bounds__(CEN_TW *CEN_TH) void census_kernel(CensusArgs a)
{
    const int H = a.H, W = a.W, pitch = a.pitch[blockIdx.z];
    const uint8_t *__restrict__ img = a.img[blockIdx.z];
    uint64_t *__restrict__ out = a.out[blockIdx.z];
    constexpr int LW = CEN_TW + 2 * CEN_RX;
    constexpr int LH = CEN_TH + 2 * CEN_RY;
    __shared__ uint8_t tile[LH][LW];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x0 = blockIdx.x * CEN_TW, y0 = blockIdx.y * CEN_TH;
    const int tid = ty * CEN_TW + tx;
    for (int i = tid; i < LH * LW; i += CEN_TW * CEN_TH) {
        int ly = i / LW, lx = i - ly * LW;
        int gy = min(max(y0 + ly - CEN_RY, 0), H - 1);
        int gx = min(max(x0 + lx - CEN_RX, 0), W - 1);
        tile[ly][lx] = img[(size_t)gy * pitch + gx];
    }
    __syncthreads();
    const int x = x0 + tx, y = y0 + ty;
    if (x >= W || y >= H) return;
    const uint32_t c = tile[ty + CEN_RY][tx + CEN_RX];
    // Neighbours 0..29 fill bits 61..32 (hi word), 30..61 fill bits 31..0.
    uint32_t hi = 0, lo = 0;
    int i = 0;
#pragma unroll
    for (int dy = -CEN_RY; dy <= CEN_RY; ++dy) {
#pragma unroll
        for (int dx = -CEN_RX; dx <= CEN_RX; ++dx) {
            if (dx == 0 && dy == 0) continue;
            uint32_t b = tile[ty + CEN_RY + dy][tx + CEN_RX + dx] < c ? 1u : 0u;
            if (i < 30)
                hi = (hi << 1) | b;
            else
                lo = (lo << 1) | b;
            ++i;
        }
    }
    out[(size_t)y * W + x] = ((uint64_t)hi << 32) | lo;
}

constexpr int COST_TP = 64;   // pixels of one row per block
constexpr int COST_NT = 256;  // threads per block

// cost[(y W + x) D + d] = popcount(base(x) ^ match(x -/+ d)), or 62 outside.
// The block's base and match census segments are staged in LDS; the block's
// output (COST_TP * D contiguous bytes) is written in coalesced 32-bit words.
__global__ __launch_bounds__(COST_NT) void cost_kernel(CostArgs a)
{
    const int H = a.H, W = a.W, D = a.D;
    const uint64_t *__restrict__ cb = a.base[blockIdx.z];
    const uint64_t *__restrict__ cm = a.match[blockIdx.z];
    uint8_t *__restrict__ cost = a.cost[blockIdx.z];
    const bool RIGHT = a.right[blockIdx.z] != 0;
    __shared__ uint64_t sb[COST_TP];
    __shared__ uint64_t sm[COST_TP + SF_DMAX];
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * COST_TP;
    const int np = min(COST_TP, W - x0);
    const uint64_t *rb = cb + (size_t)y * W;
    const uint64_t *rm = cm + (size_t)y * W;
    // Match segment: left base needs x in [x0 - D + 1, x0 + np), right base [x0, x0 + np + D - 1).
    const int mlo = RIGHT ? x0 : x0 - D + 1;
    const int mn = np + D - 1;
    for (int i = threadIdx.x; i < np; i += COST_NT) sb[i] = rb[x0 + i];
    for (int i = threadIdx.x; i < mn; i += COST_NT) {
        int gx = mlo + i;
        sm[i] = (gx >= 0 && gx < W) ? rm[gx] : 0;
    }
    __syncthreads();
    uint8_t *out = cost + ((size_t)y * W + x0) * D;
    auto one = [&](int p, int d) -> uint32_t {
        int xm = RIGHT ? x0 + p + d : x0 + p - d;
        if (xm < 0 || xm >= W) return SF_CMAX;
        return (uint32_t)__popcll(sb[p] ^ sm[xm - mlo]);
    };
    if ((D & 3) == 0) {
        const int qpp = D >> 2;  // 32-bit words per pixel
        const int nw = np * qpp;
        uint32_t *o32 = reinterpret_cast<uint32_t *>(out);
        // Power-of-two words per pixel (D = 32, 64, 128, 256): shifts, no division.
        const bool pow2 = (qpp & (qpp - 1)) == 0;
        const int sh = __ffs(qpp) - 1;
        for (int j = threadIdx.x; j < nw; j += COST_NT) {
            const int p = pow2 ? (j >> sh) : j / qpp;
            const int d = (j - p * qpp) * 4;
            uint32_t w = one(p, d) | (one(p, d + 1) << 8) | (one(p, d + 2) << 16) |
                         (one(p, d + 3) << 24);
            o32[j] = w;
        }
    } else {
        const int nb = np * D;
        for (int j = threadIdx.x; j < nb; j += COST_NT) {
            int p = j / D, d = j - p * D;
            out[j] = (uint8_t)one(p, d);
        }
    }
}

int launch_census(const CensusArgs &a, hipStream_t st)
{
    dim3 grid((a.W + CEN_TW - 1) / CEN_TW, (a.H + CEN_TH - 1) / CEN_TH, a.n);
    ProfScope prof("census", st);
    hipLaunchKernelGGL(census_kernel, grid, dim3(CEN_TW, CEN_TH), 0, st, a);
    return launch_status("census_kernel");
}

int launch_cost(const CostArgs &a, hipStream_t st)
{
    dim3 grid((a.W + COST_TP - 1) / COST_TP, a.H, a.n);
    ProfScope prof("cost", st);
    hipLaunchKernelGGL(cost_kernel, grid, dim3(COST_NT), 0, st, a);
    return launch_status("cost_kernel");
}

}  // namespace sf

using namespace sf;

extern "C" int sf_census(const uint8_t *img, int H, int W, int pitch, uint64_t *census,
                         void *stream)
{
    clear_error();
    SF_REQUIRE(img && census, SF_EINVAL, "sf_census: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_census: H and W must be positive");
    SF_REQUIRE(pitch >= W, SF_EINVAL, "sf_census: pitch < W");
    SF_REQUIRE(H <= 65535 * CEN_TH, SF_EINVAL, "sf_census: H too large");
    CensusArgs a{};
    a.img[0] = img;
    a.out[0] = census;
    a.pitch[0] = pitch;
    a.n = 1;
    a.H = H;
    a.W = W;
    return launch_census(a, as_stream(stream));
}

extern "C" int sf_cost(const uint64_t *cen_base, const uint64_t *cen_match, int H, int W, int D,
                       int base_is_right, uint8_t *cost, void *stream)
{
    clear_error();
    SF_REQUIRE(cen_base && cen_match && cost, SF_EINVAL, "sf_cost: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_cost: H and W must be positive");
    SF_REQUIRE(D >= 1 && D <= SF_DMAX, SF_EINVAL, "sf_cost: D must be in [1, 256]");
    SF_REQUIRE(H <= 65535, SF_EINVAL, "sf_cost: H > 65535");
    CostArgs a{};
    a.base[0] = cen_base;
    a.match[0] = cen_match;
    a.cost[0] = cost;
    a.right[0] = base_is_right ? 1 : 0;
    a.n = 1;
    a.H = H;
    a.W = W;
    a.D = D;
    return launch_cost(a, as_stream(stream));
}
