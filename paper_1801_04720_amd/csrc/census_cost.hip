// Census transform and Hamming matching-cost volume (the matching cost inside
// SGM, paper Sec. 3.1; the 9x7 census and Hamming distance are the workload's
// choice, the paper names no cost).
#include "lrnet_pack.hpp"
#include "sf_internal.hpp"
#include "stages.hpp"

namespace sf {

constexpr int CEN_PX = 4;                // pixels per thread: one dword of image bytes
constexpr int CEN_TX = 64;               // threads per tile row (one wave)
constexpr int CEN_TW = CEN_TX * CEN_PX;  // tile width in pixels
constexpr int CEN_TH = 4;                // tile rows (four waves)
constexpr int CEN_RX = 4;                // window half-width  (9 wide)
constexpr int CEN_RY = 3;                // window half-height (7 tall)
constexpr int CEN_LW = (CEN_TW + 2 * CEN_RX) / 4;  // LDS row length in dwords
constexpr int CEN_LH = CEN_TH + 2 * CEN_RY;        // LDS rows

// Each thread computes the census of four horizontally adjacent pixels with
// byte-parallel arithmetic.  For one window offset, the four neighbours form
// one dword n4 (an alignbyte of the thread's three row dwords) and the four
// centres another, c4.  v_lerp_u8 averages bytes with a 9-bit intermediate:
// per byte (c + (255 - n)) >> 1 >= 128 exactly when n < c, so bit 7 of each
// byte of lerp(c4, ~n4, 0) is the census bit of one pixel.  Those bits are
// shifted into eight accumulators, one per code byte (byte j of accumulator b
// is code byte b of pixel j), and a byte transpose at the end assembles the
// four 62-bit codes.  The (TH + 6) x (TW + 8) window of the tile is staged in
// LDS with clamp-to-edge.
__global__ __launch_bounds__(CEN_TX *CEN_TH) void census_kernel(CensusArgs a)
{
    if ((int)blockIdx.z == a.n) {  // the extra plane: the network's weight fragments
        const int nb = gridDim.x * gridDim.y;
        for (int s = (blockIdx.y * gridDim.x + blockIdx.x) * CEN_TH + threadIdx.y; s < FP_NSLOT; s += nb * CEN_TH)
            lrnet_pack_lane(a.pack_prm, a.pack_frag, a.pack_fl, s, threadIdx.x);
        return;
    }
    const int H = a.H, W = a.W, pitch = a.pitch[blockIdx.z];
    const uint8_t *__restrict__ img = a.img[blockIdx.z];
    uint64_t *__restrict__ out = a.out[blockIdx.z];
    __shared__ uint32_t tile[CEN_LH * CEN_LW];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x0 = blockIdx.x * CEN_TW, y0 = blockIdx.y * CEN_TH;
    const int tid = ty * CEN_TX + tx;
    // Tile byte i of LDS row r is image byte (clamp(y0 + r - RY), clamp(x0 - RX + i)).
    // Away from the left and right image edges a tile dword is assembled from
    // the two aligned dwords around its four bytes (any base or pitch
    // alignment); those reads stay inside the row because the tile starts at
    // least 7 bytes from either end.
    const bool interior = x0 >= 2 * CEN_RX && x0 + CEN_TW + 2 * CEN_RX <= W;
    if (interior) {
        for (int i = tid; i < CEN_LH * CEN_LW; i += CEN_TX * CEN_TH) {
            const int r = i / CEN_LW, c = i - r * CEN_LW;
            const int gy = min(max(y0 + r - CEN_RY, 0), H - 1);
            const uint8_t *src = img + (size_t)gy * pitch + (x0 - CEN_RX) + 4 * c;
            const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(src) & 3);
            const uint32_t *al = reinterpret_cast<const uint32_t *>(src - sh);
            const uint64_t two = (uint64_t)al[0] | ((uint64_t)al[1] << 32);
            tile[i] = (uint32_t)(two >> (8 * sh));
        }
    } else {
        uint8_t *tb = reinterpret_cast<uint8_t *>(tile);
        for (int i = tid; i < CEN_LH * CEN_LW * 4; i += CEN_TX * CEN_TH) {
            const int r = i / (CEN_LW * 4), c = i - r * (CEN_LW * 4);
            const int gy = min(max(y0 + r - CEN_RY, 0), H - 1);
            const int gx = min(max(x0 - CEN_RX + c, 0), W - 1);
            tb[i] = img[(size_t)gy * pitch + gx];
        }
    }
    __syncthreads();
    const int x = x0 + CEN_PX * tx, y = y0 + ty;
    if (x >= W || y >= H) return;
    // Row dword k of window row r holds bytes x - 4 + 4k .. x - 1 + 4k.
    uint32_t w[2 * CEN_RY + 1][3];
#pragma unroll
    for (int r = 0; r < 2 * CEN_RY + 1; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) w[r][k] = tile[(ty + r) * CEN_LW + tx + k];
    const uint32_t c4 = w[CEN_RY][1];
    uint32_t acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[b] = 0;
    // Neighbour k (row-major, centre skipped) is code bit 61 - k.  Visiting k
    // downwards fills every code byte from its lowest bit up, so each new bit
    // enters at bit 7 of its byte while the earlier ones move down.
    int k = 61;
#pragma unroll
    for (int dy = CEN_RY; dy >= -CEN_RY; --dy) {
        const uint32_t n0 = ~w[dy + CEN_RY][0], n1 = ~w[dy + CEN_RY][1], n2 = ~w[dy + CEN_RY][2];
#pragma unroll
        for (int dx = CEN_RX; dx >= -CEN_RX; --dx) {
            if (dx == 0 && dy == 0) continue;
            const int s = dx + CEN_RX;  // byte offset of the neighbours within x - 4 .. x + 7
            const uint32_t lo = s < 4 ? n0 : s < 8 ? n1 : n2, hi = s < 4 ? n1 : n2;
            const uint32_t nn = (s & 3) == 0 ? lo : (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * (s & 3)));
            const uint32_t t = __builtin_amdgcn_lerp(c4, nn, 0u);
            const int b = (61 - k) >> 3;
            acc[b] = (t & 0x80808080u) | ((acc[b] >> 1) & 0x7f7f7f7fu);
            --k;
        }
    }
    acc[7] = (acc[7] >> 2) & 0x3f3f3f3fu;  // bits 56..61 of the code; 62 and 63 are zero
    uint32_t lo[CEN_PX], hi[CEN_PX];
#pragma unroll
    for (int j = 0; j < CEN_PX; ++j) {
        const int sh = 8 * j;
        lo[j] = ((acc[0] >> sh) & 0xffu) | (((acc[1] >> sh) & 0xffu) << 8) |
                (((acc[2] >> sh) & 0xffu) << 16) | (((acc[3] >> sh) & 0xffu) << 24);
        hi[j] = ((acc[4] >> sh) & 0xffu) | (((acc[5] >> sh) & 0xffu) << 8) |
                (((acc[6] >> sh) & 0xffu) << 16) | (((acc[7] >> sh) & 0xffu) << 24);
    }
    uint64_t *o = out + (size_t)y * W + x;
    if (x + CEN_PX <= W && (reinterpret_cast<uintptr_t>(o) & 15) == 0) {
        reinterpret_cast<uint4 *>(o)[0] = make_uint4(lo[0], hi[0], lo[1], hi[1]);
        reinterpret_cast<uint4 *>(o)[1] = make_uint4(lo[2], hi[2], lo[3], hi[3]);
    } else {
#pragma unroll
        for (int j = 0; j < CEN_PX; ++j)
            if (x + j < W) o[j] = ((uint64_t)hi[j] << 32) | lo[j];
    }
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
    if (a.vec == 4) {
        const int qpp = D >> 2;  // 32-bit words per pixel
        const int nw = np * qpp;
        uint32_t *o32 = reinterpret_cast<uint32_t *>(out);
        for (int j = threadIdx.x; j < nw; j += COST_NT) {
            const int p = j / qpp;
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

// 16-byte path (D a multiple of 16, aligned output).  Thread (chunk c, run j)
// produces disparities [16c, 16c + 16) of CV_R consecutive pixels; the
// CV_R + 15 match census words it needs are read once from LDS into registers
// (a sliding window) instead of once per disparity.  The chunk index runs
// fastest, so the threads of one pixel write its D bytes contiguously.
// LDS index i is stored at i + i/8: a wave's reads hit indices 8k + const,
// which this maps to distinct banks.
constexpr int CV_NT = 256;  // threads per block
constexpr int CV_R = 8;     // consecutive pixels per thread

__host__ __device__ __forceinline__ int cv_swz(int i) { return i + (i >> 3); }

__device__ __forceinline__ uint32_t hamming(uint64_t b, uint64_t m)
{
    const uint64_t x = b ^ m;
    return (uint32_t)__popc((uint32_t)x) + (uint32_t)__popc((uint32_t)(x >> 32));
}

// 16 six-bit values (LSB first) packed into three dwords.
__device__ __forceinline__ uint3 pack6x16(const uint32_t (&v)[16])
{
    uint32_t p[3] = {0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int bit = 6 * e, w = bit >> 5, s = bit & 31;
        p[w] |= v[e] << s;
        if (s > 26) p[w + 1] |= v[e] >> (32 - s);  // the field crosses into the next dword
    }
    return make_uint3(p[0], p[1], p[2]);
}

// PACK: write the 16 costs of the run as 6-bit fields (12 bytes at byte 12c of
// the pixel's 0.75 D bytes); otherwise as 16 bytes at byte 16c of its D bytes.
template <bool RIGHT, bool EDGE, bool PACK = false>
__device__ __forceinline__ void cost_run16(const uint64_t *sb, const uint64_t *sm, int j, int c,
                                           int x0, int W, int D, uint8_t *row)
{
    // Window word k holds the match census at LDS index  j R + 16c + k (right
    // base; element (r, e) uses k = r + e) or  j R + D - 1 - 16c - 15 + k
    // (left base; element (r, e) uses k = r - e + 15).
    uint64_t win[CV_R + 15];
    const int w0 = RIGHT ? j * CV_R + 16 * c : j * CV_R + D - 16 - 16 * c;
#pragma unroll
    for (int k = 0; k < CV_R + 15; ++k) win[k] = sm[cv_swz(w0 + k)];
#pragma unroll
    for (int r = 0; r < CV_R; ++r) {
        const int xl = j * CV_R + r;  // block-local pixel
        const int x = x0 + xl;
        const uint64_t b = sb[cv_swz(xl)];
        uint32_t v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            v[e] = hamming(b, win[RIGHT ? r + e : r - e + 15]);
            if (EDGE) {
                const int d = 16 * c + e;
                const bool out = RIGHT ? (x + d >= W) : (x - d < 0);
                v[e] = out ? (uint32_t)SF_CMAX : v[e];
            }
        }
        if (x >= W) continue;
        if constexpr (PACK) {
            *reinterpret_cast<uint3 *>(row + (size_t)xl * (3 * D / 4) + 12 * c) = pack6x16(v);
        } else {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                w[q] = v[4 * q] | (v[4 * q + 1] << 8) | (v[4 * q + 2] << 16) | (v[4 * q + 3] << 24);
            reinterpret_cast<uint4 *>(row + (size_t)xl * D)[c] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

__global__ __launch_bounds__(CV_NT) void cost16_kernel(CostArgs a)
{
    extern __shared__ uint64_t cv_lds[];
    const int H = a.H, W = a.W, D = a.D;
    (void)H;
    const uint64_t *__restrict__ cb = a.base[blockIdx.z];
    const uint64_t *__restrict__ cm = a.match[blockIdx.z];
    const bool RIGHT = a.right[blockIdx.z] != 0;
    const int cpp = D >> 4;           // 16-disparity chunks per pixel
    const int runs = CV_NT / cpp;     // pixel runs per block
    const int TP = runs * CV_R;       // pixels per block
    const int y = blockIdx.y, x0 = blockIdx.x * TP;
    const int mn = TP + D - 1;        // match words: x0 - D + 1 .. x0 + TP - 1 (left), x0 .. x0 + TP + D - 2 (right)
    const int mlo = RIGHT ? x0 : x0 - D + 1;
    uint64_t *sb = cv_lds;
    uint64_t *sm = cv_lds + cv_swz(TP - 1) + 1;
    const uint64_t *rb = cb + (size_t)y * W;
    const uint64_t *rm = cm + (size_t)y * W;
    for (int i = threadIdx.x; i < TP; i += CV_NT) {
        const int gx = x0 + i;
        sb[cv_swz(i)] = gx < W ? rb[gx] : 0;
    }
    for (int i = threadIdx.x; i < mn; i += CV_NT) {
        const int gx = mlo + i;
        sm[cv_swz(i)] = (gx >= 0 && gx < W) ? rm[gx] : 0;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int c = t % cpp, j = t / cpp;
    if (j >= runs) return;
    const bool edge = RIGHT ? (x0 + TP + D - 2 >= W) : (x0 < D - 1);
    if (a.packed) {
        uint8_t *row = a.cost[blockIdx.z] + ((size_t)y * W + x0) * (3 * D / 4);
        if (RIGHT)
            edge ? cost_run16<true, true, true>(sb, sm, j, c, x0, W, D, row)
                 : cost_run16<true, false, true>(sb, sm, j, c, x0, W, D, row);
        else
            edge ? cost_run16<false, true, true>(sb, sm, j, c, x0, W, D, row)
                 : cost_run16<false, false, true>(sb, sm, j, c, x0, W, D, row);
    } else {
        uint8_t *row = a.cost[blockIdx.z] + ((size_t)y * W + x0) * D;
        if (RIGHT)
            edge ? cost_run16<true, true>(sb, sm, j, c, x0, W, D, row)
                 : cost_run16<true, false>(sb, sm, j, c, x0, W, D, row);
        else
            edge ? cost_run16<false, true>(sb, sm, j, c, x0, W, D, row)
                 : cost_run16<false, false>(sb, sm, j, c, x0, W, D, row);
    }
}

// Pixels per block and dynamic LDS bytes of cost16_kernel.
static inline int cv_tile(int D) { return (CV_NT / (D >> 4)) * CV_R; }
static inline size_t cv_lds_bytes(int D)
{
    const int TP = cv_tile(D);
    return (size_t)(cv_swz(TP - 1) + 1 + cv_swz(TP + D - 2) + 1) * sizeof(uint64_t);
}

int launch_census(const CensusArgs &a, hipStream_t st)
{
    if (a.pack_prm && a.n >= STAGE_MAXV) return fail(SF_EINVAL, "launch_census: no plane left for packing");
    dim3 grid((a.W + CEN_TW - 1) / CEN_TW, (a.H + CEN_TH - 1) / CEN_TH, a.n + (a.pack_prm ? 1 : 0));
    ProfScope prof("census", st);
    hipLaunchKernelGGL(census_kernel, grid, dim3(CEN_TX, CEN_TH), 0, st, a);
    return launch_status("census_kernel");
}

int launch_cost(const CostArgs &args, hipStream_t st)
{
    CostArgs a = args;
    uintptr_t ptr_bits = 0;
    for (int i = 0; i < a.n; ++i) ptr_bits |= reinterpret_cast<uintptr_t>(a.cost[i]);
    a.vec = ((a.D & 15) == 0 && (ptr_bits & 15) == 0) ? 16 : ((a.D & 3) == 0 && (ptr_bits & 3) == 0) ? 4 : 1;
    if (a.packed) {
        if (!cost_packable(a.D) || (ptr_bits & 3) != 0)
            return fail(SF_EINVAL, "launch_cost: packed costs need D = 128 or 256 and 4-byte aligned volumes");
        a.vec = 16;  // the 16-disparity-run kernel writes the packed runs
    }
    ProfScope prof("cost", st);
    if (a.vec == 16) {
        const int TP = cv_tile(a.D);
        dim3 grid((a.W + TP - 1) / TP, a.H, a.n);
        hipLaunchKernelGGL(cost16_kernel, grid, dim3(CV_NT), cv_lds_bytes(a.D), st, a);
        return launch_status("cost16_kernel");
    }
    dim3 grid((a.W + COST_TP - 1) / COST_TP, a.H, a.n);
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
