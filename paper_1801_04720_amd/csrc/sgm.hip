// Semi-global path aggregation (paper Sec. 3.1: eight paths radiating from
// each pixel; the per-path recurrence with penalties P1 / P2 of the cited SGM
// method).
//
// Work decomposition (CDNA wave64):
//   * one "path chain" = one scanline of one direction, walked from the image
//     edge where its predecessor leaves the image;
//   * a chain is owned by one 16-lane DPP row; lane j of the row holds the K =
//     D/16 disparities [jK, jK+K) as K/2 packed u16 pairs, interleaved: pair i
//     holds d = jK + i (low half) and d = jK + K/2 + i (high half).  Then the
//     d-1 neighbours of pair i are exactly pair i-1 and the d+1 neighbours pair
//     i+1; only the two end pairs need a v_alignbit with one row_shr / row_shl
//     DPP move across lanes.  min_k Lr(p-r, k) is a 4-step DPP butterfly inside
//     the row (quad_perm, half-mirror, mirror);
//   * slabs keep each lane's K bytes in the same interleaved order (byte 2i =
//     pair i low, byte 2i+1 = pair i high): position e of lane j's chunk holds
//     d = jK + e/2 + (e%2) K/2.  Their consumers map positions back to d.
//   * a wave carries 4 chains, a 256-thread block 16.
//   * Lr needs at most 62 + P2 <= 255 (u8) when P2 <= 193: each direction's
//     Lr is then streamed to its own u8 slab and the consumer sums the slabs
//     (a separate pass into S, or on the fly inside WTA).  Otherwise Lr is added
//     into a zeroed S with packed 32-bit atomics (each u16 half stays below
//     8 (62 + P2) < 2^16, so no carry crosses halves).
//
//   * intensity-adaptive P2 (a variant of the cited method): the chain also
//     streams its base-image bytes I(p) (prefetched with the costs) and uses
//     max(P1, floor(P2 / |I(p) - I(p - r)|)) at each step (P2 where the step is
//     flat); the quotient is a float reciprocal product corrected by one
//     integer step either way, which is exact for P2 <= 8000, g <= 255.
//
// Two launch shapes share the chain code:
//   * sgm_paths_kernel: one view, the block index enumerates its chains;
//   * sgm_tasks_kernel: many views (the four of a scene-flow frame, or a batch
//     of uneven stereo pairs) from a task table sorted longest chains first,
//     each block one task of up to 16 chains of one view and direction, K
//     chosen per task; optionally persistent, pulling tasks from a counter.
#include <type_traits>

#include "sf_check.hpp"
#include "sf_internal.hpp"
#include "sgm_tasks.hpp"

SF_CHECK_TU(sgm)

namespace sf {

constexpr int SGM_NT = 256;              // threads per block
constexpr int SGM_CPB = SGM_NT / 16;     // chains per block
constexpr uint32_t SGM_SENT = 0x7FFF7FFFu;  // "no neighbour" value, never the minimum

__constant__ int c_dir[8][2] = {{+1, 0}, {-1, 0}, {0, +1}, {0, -1},
                                {+1, +1}, {-1, +1}, {+1, -1}, {-1, -1}};

struct PathTable {
    int ndir;
    int dir[8];
    int n[8];          // chains of each selected direction
    int off[9];        // prefix sums of the chain counts rounded up to whole blocks, so
                       // that every block (and wave) walks chains of one direction
};

// Start pixel and length of chain l of direction r.
__device__ __forceinline__ void chain_geometry(int r, int l, int H, int W, int &x, int &y, int &len)
{
    const int rx = c_dir[r][0], ry = c_dir[r][1];
    if (ry == 0) {
        x = rx > 0 ? 0 : W - 1;
        y = l;
        len = W;
    } else if (rx == 0) {
        x = l;
        y = ry > 0 ? 0 : H - 1;
        len = H;
    } else {
        const int xe = rx > 0 ? 0 : W - 1, ye = ry > 0 ? 0 : H - 1;
        if (l < H) {
            x = xe;
            y = ry > 0 ? l : H - 1 - l;
        } else {
            const int k = l - H;  // 0 .. W-2, skipping the corner column
            x = rx > 0 ? k + 1 : W - 2 - k;
            y = ye;
        }
        const int nx = rx > 0 ? W - x : x + 1;
        const int ny = ry > 0 ? H - y : y + 1;
        len = min(nx, ny);
    }
}

// Raw cost bytes of one lane for one pixel, and their unpacking into u16 pairs.
template <int K>
struct CostRaw {
    static constexpr int N = (K % 4 == 0) ? K / 4 : K / 2;
    uint32_t w[N];
};

template <int K>
__device__ __forceinline__ void load_raw(const uint8_t *p, CostRaw<K> &r)
{
    if constexpr (K % 16 == 0) {
#pragma unroll
        for (int q = 0; q < K / 16; ++q) {
            uint4 v = reinterpret_cast<const uint4 *>(p)[q];
            r.w[4 * q + 0] = v.x;
            r.w[4 * q + 1] = v.y;
            r.w[4 * q + 2] = v.z;
            r.w[4 * q + 3] = v.w;
        }
    } else if constexpr (K % 8 == 0) {
#pragma unroll
        for (int q = 0; q < K / 8; ++q) {
            uint2 v = reinterpret_cast<const uint2 *>(p)[q];
            r.w[2 * q + 0] = v.x;
            r.w[2 * q + 1] = v.y;
        }
    } else if constexpr (K % 4 == 0) {
#pragma unroll
        for (int q = 0; q < K / 4; ++q) r.w[q] = reinterpret_cast<const uint32_t *>(p)[q];
    } else {
#pragma unroll
        for (int q = 0; q < K / 2; ++q) r.w[q] = reinterpret_cast<const uint16_t *>(p)[q];
    }
}

// The same through a raw buffer resource: 32-bit offsets, and offsets past the
// volume (steps beyond a chain's end) read zeros instead of faulting.
constexpr int SGM_RSRC_WORD3 = 0x00020000;  // raw buffer, gfx9-family data format

template <int K>
__device__ __forceinline__ void load_raw_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, CostRaw<K> &r)
{
    if constexpr (K % 16 == 0) {
#pragma unroll
        for (int q = 0; q < K / 16; ++q) {
            const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16 * q), 0, 0));
            r.w[4 * q + 0] = v.x;
            r.w[4 * q + 1] = v.y;
            r.w[4 * q + 2] = v.z;
            r.w[4 * q + 3] = v.w;
        }
    } else if constexpr (K % 8 == 0) {
#pragma unroll
        for (int q = 0; q < K / 8; ++q) {
            const u32x2 v = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(off + 8 * q), 0, 0));
            r.w[2 * q + 0] = v.x;
            r.w[2 * q + 1] = v.y;
        }
    } else if constexpr (K % 4 == 0) {
#pragma unroll
        for (int q = 0; q < K / 4; ++q) r.w[q] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + 4 * q), 0, 0);
    } else {
#pragma unroll
        for (int q = 0; q < K / 2; ++q)
            r.w[q] = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(rs, (int)(off + 2 * q), 0, 0);
    }
}

// Cost bytes (d order) -> interleaved u16 pairs: pair i = (d = jK + i, d = jK + K/2 + i).
template <int K>
__device__ __forceinline__ void unpack(const CostRaw<K> &r, uint32_t (&c)[K / 2])
{
#pragma unroll
    for (int i = 0; i < K / 2; ++i) {
        const int lo = i, hi = K / 2 + i;
        if constexpr (K % 4 == 0) {
            const uint32_t sel = (uint32_t)(lo % 4) | (0x0cu << 8) | ((uint32_t)(4 + hi % 4) << 16) |
                                 (0x0cu << 24);
            c[i] = __builtin_amdgcn_perm(r.w[hi / 4], r.w[lo / 4], sel);
        } else {
            const uint32_t sel = (uint32_t)(lo % 2) | (0x0cu << 8) | ((uint32_t)(4 + hi % 2) << 16) |
                                 (0x0cu << 24);
            c[i] = __builtin_amdgcn_perm(r.w[hi / 2], r.w[lo / 2], sel);
        }
    }
}

template <int K, bool ATOMIC>
__device__ __forceinline__ void emit(const uint32_t (&L)[K / 2], uint8_t *slab_px, uint16_t *s_px)
{
    if constexpr (ATOMIC) {
        // Back to d order: word m holds d = jK + 2m and jK + 2m + 1; relative d
        // below K/2 sits in the low half of pair d, the rest in the high half of
        // pair d - K/2.
        uint32_t *s32 = reinterpret_cast<uint32_t *>(s_px);
        constexpr int NP = K / 2;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            const int d0 = 2 * m, d1 = 2 * m + 1;
            const int p0 = d0 < NP ? d0 : d0 - NP, p1 = d1 < NP ? d1 : d1 - NP;
            const uint32_t sel = (d0 < NP ? 0x0100u : 0x0302u) | (d1 < NP ? 0x05040000u : 0x07060000u);
            atomicAdd(s32 + m, __builtin_amdgcn_perm(L[p1], L[p0], sel));
        }
    } else {
        // Low byte of each u16 half -> K consecutive bytes.
        if constexpr (K % 4 == 0) {
            uint32_t b[K / 4];
#pragma unroll
            for (int q = 0; q < K / 4; ++q)
                b[q] = __builtin_amdgcn_perm(L[2 * q + 1], L[2 * q], 0x06040200u);
            // Slabs are written once and read once, much later: stream them past
            // the caches (non-temporal) so the cost volumes stay cached.
            if constexpr (K % 16 == 0) {
#pragma unroll
                for (int q = 0; q < K / 16; ++q)
                    __builtin_nontemporal_store(
                        u32x4{b[4 * q], b[4 * q + 1], b[4 * q + 2], b[4 * q + 3]},
                        reinterpret_cast<u32x4 *>(slab_px) + q);
            } else if constexpr (K % 8 == 0) {
#pragma unroll
                for (int q = 0; q < K / 8; ++q)
                    __builtin_nontemporal_store(u32x2{b[2 * q], b[2 * q + 1]},
                                                reinterpret_cast<u32x2 *>(slab_px) + q);
            } else {
#pragma unroll
                for (int q = 0; q < K / 4; ++q)
                    __builtin_nontemporal_store(b[q], reinterpret_cast<uint32_t *>(slab_px) + q);
            }
        } else {
#pragma unroll
            for (int q = 0; q < K / 2; ++q)
                reinterpret_cast<uint16_t *>(slab_px)[q] =
                    (uint16_t)__builtin_amdgcn_perm(0u, L[q], 0x0c0c0200u);
        }
    }
}

// Slab store through a buffer resource (32-bit offsets), non-temporal: slabs are
// written once and read once, much later, so they should not evict the cost
// volumes from the caches.
template <int K>
__device__ __forceinline__ void emit_buf(const uint32_t (&L)[K / 2], __amdgpu_buffer_rsrc_t rs,
                                         uint32_t off)
{
    constexpr int NT = 2;  // non-temporal
    if constexpr (K % 4 == 0) {
        uint32_t b[K / 4];
#pragma unroll
        for (int q = 0; q < K / 4; ++q) b[q] = __builtin_amdgcn_perm(L[2 * q + 1], L[2 * q], 0x06040200u);
        if constexpr (K % 16 == 0) {
#pragma unroll
            for (int q = 0; q < K / 16; ++q)
                __builtin_amdgcn_raw_buffer_store_b128(u32x4{b[4 * q], b[4 * q + 1], b[4 * q + 2], b[4 * q + 3]},
                                                       rs, (int)(off + 16 * q), 0, NT);
        } else if constexpr (K % 8 == 0) {
#pragma unroll
            for (int q = 0; q < K / 8; ++q)
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{b[2 * q], b[2 * q + 1]}, rs, (int)(off + 8 * q), 0, NT);
        } else {
#pragma unroll
            for (int q = 0; q < K / 4; ++q) __builtin_amdgcn_raw_buffer_store_b32(b[q], rs, (int)(off + 4 * q), 0, NT);
        }
    } else {
#pragma unroll
        for (int q = 0; q < K / 2; ++q)
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)__builtin_amdgcn_perm(0u, L[q], 0x0c0c0200u), rs,
                                                  (int)(off + 2 * q), 0, NT);
    }
}

// Packed costs (6 bits each, the frame and batch paths at D = 128 or 256):
// lane j's K costs d = jK .. jK + K - 1 are K consecutive 6-bit fields.  For
// K = 8 they are the 6 bytes at byte 6j of the pixel's 96; the lane reads the
// 8 aligned bytes at 12 (j / 2) + 4 (j % 2) and drops 16 bits when j is odd.
// For K = 16 they are the 12 bytes at byte 12j of the pixel's 192.
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));

template <int K>
struct CostPk {
    static_assert(K == 8 || K == 16, "packed costs need K = 8 or 16");
    uint32_t w[K == 8 ? 2 : 3];
};

template <int K>
__device__ __forceinline__ uint32_t pk_lane_off(int j)
{
    return K == 8 ? (uint32_t)(12 * (j >> 1) + 4 * (j & 1)) : (uint32_t)(12 * j);
}

template <int K>
__device__ __forceinline__ void load_pk_buf(__amdgpu_buffer_rsrc_t rs, uint32_t off, CostPk<K> &r)
{
    if constexpr (K == 8) {
        const u32x2 v = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
        r.w[0] = v.x;
        r.w[1] = v.y;
    } else {
        const u32x3 v = __builtin_bit_cast(u32x3, __builtin_amdgcn_raw_buffer_load_b96(rs, (int)off, 0, 0));
        r.w[0] = v.x;
        r.w[1] = v.y;
        r.w[2] = v.z;
    }
}

// Field e (bits 6e .. 6e + 5) of a little-endian multiword (e a constant).
template <int NW>
__device__ __forceinline__ uint32_t field6(const uint32_t (&w)[NW], int e)
{
    const int bit = 6 * e, k = bit >> 5, s = bit & 31;
    if (s <= 26) return (w[k] >> s) & 63u;
    return __builtin_amdgcn_alignbit(w[k + 1], w[k], s) & 63u;
}

// Packed costs -> interleaved u16 pairs: pair i = (d = jK + i, d = jK + K/2 + i).
template <int K>
__device__ __forceinline__ void unpack_pk(const CostPk<K> &r, int j, uint32_t (&c)[K / 2])
{
    if constexpr (K == 8) {
        const uint32_t sh = 16u * (uint32_t)(j & 1);
        const uint32_t f[2] = {__builtin_amdgcn_alignbit(r.w[1], r.w[0], sh), r.w[1] >> sh};
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = field6<2>(f, i) | (field6<2>(f, i + 4) << 16);
    } else {
        (void)j;
#pragma unroll
        for (int i = 0; i < 8; ++i) c[i] = field6<3>(r.w, i) | (field6<3>(r.w, i + 8) << 16);
    }
}

// Census mode (no cost volume): the lane computes its K costs of a pixel from
// the base pixel's census word and the K match words, C = popcount(base ^
// match), SF_CMAX where the match pixel lies outside the image.  CEN = 1: left
// base, match pixel x - d; CEN = 2: right base, match pixel x + d.  The match
// words of relative disparity e = 0 .. K-1 are K consecutive words of the row,
// fetched as K/2 16-byte loads: load q holds e = 2q, 2q + 1 (right base,
// ascending x) or e = 2q + 1, 2q (left base, descending x).  A left-base load
// that would start one word before the array (x - d = 0 on row 0 for e = 2q)
// starts at the array instead (the buffer's range check would drop both words
// otherwise), so e = 2q then sits in the first half; that happens only where
// some lane has a match pixel outside the image, the slow path below.
template <int K>
struct CenRaw {
    uint32_t b[2];      // base census word (low, high)
    uint32_t m[2 * K];  // match words as loaded, 4 per 16-byte load
    int lim;            // the match pixel of relative disparity e is inside iff e <= lim
    int row0;           // the pixel is on row 0 (left base: loads may have been moved)
};

// Words of relative disparity e in the load order (no moved load).
template <int K, int CEN>
__device__ __forceinline__ int cen_slot(int e)
{
    const int q = e >> 1, odd = e & 1;
    return 4 * q + ((CEN == 1) == (odd != 0) ? 0 : 2);
}

template <int K>
__device__ __forceinline__ uint32_t cen_hamming(const CenRaw<K> &r, int slot)
{
    return (uint32_t)(__builtin_popcount(r.b[0] ^ r.m[slot]) + __builtin_popcount(r.b[1] ^ r.m[slot + 1]));
}

template <int K, int CEN>
__device__ __forceinline__ uint32_t cen_cost(const CenRaw<K> &r, int e)
{
    int slot = cen_slot<K, CEN>(e);
    if (CEN == 1 && (e & 1) == 0) {
        // Moved load: its start offset was negative, i.e. row 0 and x - jK - e - 1 < 0.
        if (r.row0 && r.lim < e + 1) slot -= 2;
    }
    const uint32_t c = cen_hamming<K>(r, slot);
    return e <= r.lim ? c : (uint32_t)SF_CMAX;
}

// Census words -> interleaved u16 pairs: pair i = (e = i, e = K/2 + i).  Where
// no lane of the wave has a match pixel outside the image (all but the first
// D columns of a left base, the last D of a right base) the range tests are
// skipped.
template <int K, int CEN>
__device__ __forceinline__ void unpack_cen(const CenRaw<K> &r, uint32_t (&c)[K / 2])
{
    if (__builtin_amdgcn_ballot_w64(r.lim < K - 1) == 0) {
#pragma unroll
        for (int i = 0; i < K / 2; ++i)
            c[i] = cen_hamming<K>(r, cen_slot<K, CEN>(i)) | (cen_hamming<K>(r, cen_slot<K, CEN>(K / 2 + i)) << 16);
    } else {
#pragma unroll
        for (int i = 0; i < K / 2; ++i) c[i] = cen_cost<K, CEN>(r, i) | (cen_cost<K, CEN>(r, K / 2 + i) << 16);
    }
}

// Default prefetch depth (steps) of the cost stream of one chain.
constexpr int SGM_U = 8;
// Prefetch depth in census mode (each step holds 2 K + 3 registers).
template <int K>
constexpr int sgm_cen_u() { return K <= 8 ? 2 : 1; }

// Walk chain l of direction r with the 16 lanes of this DPP row (lane j).
// cost: [H][W][D]; slab: this direction's [H][W][D] u8 slab (ATOMIC == false)
// or S [H][W][D] u16 (ATOMIC == true).
// CEN != 0: costs from the census words cen_b (base) and cen_m (match) instead
// of the cost volume (unused then).
template <int K, bool ATOMIC, int U = SGM_U, bool ADAPT = false, bool PACK = false, int CEN = 0>
__device__ __forceinline__ void sgm_chain(const uint8_t *__restrict__ cost, uint8_t *__restrict__ slab,
                                          uint16_t *__restrict__ S, int H, int W, int P1, int P2,
                                          int r, int l, int j, const uint8_t *img = nullptr,
                                          int pitch = 0, const uint64_t *cen_b = nullptr,
                                          const uint64_t *cen_m = nullptr)
{
    static_assert(CEN == 0 || (!ADAPT && !PACK), "census mode takes neither packed costs nor adaptive P2");
    constexpr int D = 16 * K;
    constexpr int NP = K / 2;
    constexpr int CPX = PACK ? 3 * D / 4 : D;  // cost bytes per pixel
    int x, y, len;
    chain_geometry(r, l, H, W, x, y, len);
    const int rx = c_dir[r][0], ry = c_dir[r][1];
    // Byte steps along the chain in the [H][W][D] output volumes and the cost volume.
    const ptrdiff_t bstep = ((ptrdiff_t)ry * W + rx) * D;
    const size_t b0 = ((size_t)y * W + x) * D + (size_t)j * K;
    const ptrdiff_t cstep = ((ptrdiff_t)ry * W + rx) * CPX;
    const size_t c0 = ((size_t)y * W + x) * CPX + (PACK ? (size_t)pk_lane_off<PACK ? K : 8>(j) : (size_t)j * K);
    // Cost volume through a buffer resource (the volume is < 2^31 bytes).
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(cost), (short)0, (int)((size_t)H * W * CPX), SGM_RSRC_WORD3);
    uint32_t ld = (uint32_t)c0;                                  // next cost load (offset)
    const __amdgpu_buffer_rsrc_t rs_out = __builtin_amdgcn_make_buffer_rsrc(
        ATOMIC ? (void *)S : (void *)slab, (short)0, (int)((size_t)H * W * D), SGM_RSRC_WORD3);
    uint32_t st = (uint32_t)b0;                                  // next slab store (offset)
    uint16_t *stS = ATOMIC ? S + b0 : nullptr;                   // next S update
    // Base image along the chain (adaptive P2 only), same out-of-range rule.
    const __amdgpu_buffer_rsrc_t rs_img = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(ADAPT ? img : cost), (short)0, ADAPT ? (int)((size_t)H * pitch) : 0,
        SGM_RSRC_WORD3);
    uint32_t ild = ADAPT ? (uint32_t)(y * pitch + x) : 0u;
    const uint32_t istep = ADAPT ? (uint32_t)(ry * pitch + rx) : 0u;
    // Census words (census mode): byte offsets of the base word and of the
    // match word of e = 0 at the next fetched step.  Offsets left of a row's
    // start or past the array wrap or run beyond the buffer, which reads zeros;
    // those costs are replaced by SF_CMAX (lim) anyway.
    const int cbytes = CEN ? (int)((size_t)H * W * 8) : 0;
    const __amdgpu_buffer_rsrc_t rs_cb = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint64_t *>(CEN ? cen_b : nullptr), (short)0, cbytes, SGM_RSRC_WORD3);
    const __amdgpu_buffer_rsrc_t rs_cm = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint64_t *>(CEN ? cen_m : nullptr), (short)0, cbytes, SGM_RSRC_WORD3);
    const uint32_t cwstep = 8u * (uint32_t)(ry * W + rx);
    uint32_t cbo = CEN ? 8u * (uint32_t)(y * W + x) : 0u;
    uint32_t cmo = CEN ? 8u * (uint32_t)(y * W + x + (CEN == 1 ? -j * K : j * K)) : 0u;
    int cx = x;
    const float fP2 = (float)P2;
    uint32_t prevI = 0;

    const u16x2 vP1 = (u16x2)((unsigned short)P1);
    // Path start: with Lr(p - r, .) = 0 and M = 0 the recurrence gives exactly
    // Lr(p, d) = C(p, d) (every candidate of the min is >= 0 and Lr(d) = 0), so
    // the first step needs no special case.
    uint32_t L[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) L[i] = 0;
    uint32_t M = 0;
    // Loop-carried DPP destinations: the lanes with no source in the row (lane 0
    // for row_shr, lane 15 for row_shl) keep the "no neighbour" value forever.
    uint32_t below = SGM_SENT, above = SGM_SENT;
    // Steps past the end of this chain (other chains of the wave may be longer)
    // load whatever the buffer holds there (zeros beyond it) and store nothing.
    using Raw = std::conditional_t<(CEN != 0), CenRaw<K>,
                                   std::conditional_t<PACK, CostPk<PACK ? K : 8>, CostRaw<K>>>;
    auto fetch = [&](int t0, Raw(&buf)[U], uint32_t(&ib)[U]) {
        (void)t0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (CEN != 0) {
                const u32x2 bw = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs_cb, (int)cbo, 0, 0));
                buf[u].b[0] = bw.x;
                buf[u].b[1] = bw.y;
#pragma unroll
                for (int q = 0; q < K / 2; ++q) {
                    int o;
                    if constexpr (CEN == 1)
                        o = max((int)(cmo - 16u * (uint32_t)q - 8u), 0);  // moved load (see CenRaw)
                    else
                        o = (int)(cmo + 16u * (uint32_t)q);
                    const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs_cm, o, 0, 0));
                    buf[u].m[4 * q + 0] = v.x;
                    buf[u].m[4 * q + 1] = v.y;
                    buf[u].m[4 * q + 2] = v.z;
                    buf[u].m[4 * q + 3] = v.w;
                }
                buf[u].lim = CEN == 1 ? cx - j * K : W - 1 - cx - j * K;
                buf[u].row0 = cbo < 8u * (uint32_t)W;
                cbo += cwstep;
                cmo += cwstep;
                cx += rx;
            } else if constexpr (PACK) {
                if (t0 + u < len) SF_BOUNDS((size_t)ld + (K == 8 ? 8 : 12) <= (size_t)H * W * CPX, CHK_SGM_COST);
                load_pk_buf<K>(rs, ld, buf[u]);
            } else {
                if (t0 + u < len) SF_BOUNDS((size_t)ld + K <= (size_t)H * W * CPX, CHK_SGM_COST);
                load_raw_buf<K>(rs, ld, buf[u]);
            }
            ld += (uint32_t)cstep;
            if constexpr (ADAPT) {
                ib[u] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs_img, (int)ild, 0, 0);
                ild += istep;
            } else {
                ib[u] = 0;
            }
        }
    };
    auto step = [&](int t, const Raw &raw, uint32_t inten) {
        uint32_t c[NP];
        if constexpr (CEN != 0)
            unpack_cen<K, CEN>(raw, c);
        else if constexpr (PACK)
            unpack_pk<K>(raw, j, c);
        else
            unpack<K>(raw, c);
        below = dpp_fill<DPP_ROW_SHR1>(below, L[NP - 1]);
        above = dpp_fill<DPP_ROW_SHL1>(above, L[0]);
        uint32_t p2 = (uint32_t)P2;
        if constexpr (ADAPT) {
            // At the path start (L = 0, M = 0) any penalty gives Lr = C, so the
            // first step needs no predecessor intensity.
            const int gd = (int)inten - (int)prevI;
            const int g = gd < 0 ? -gd : gd;
            prevI = inten;
            const int g1 = g > 0 ? g : 1;
            int q = (int)(fP2 * __builtin_amdgcn_rcpf((float)g1));
            const int rem = P2 - q * g1;
            q += (rem >= g1 ? 1 : 0) - (rem < 0 ? 1 : 0);
            p2 = g == 0 ? (uint32_t)P2 : (uint32_t)(q > P1 ? q : P1);
        }
        (void)inten;
        const u16x2 vM = (u16x2)((unsigned short)M);
        const u16x2 vMP2 = (u16x2)((unsigned short)(M + p2));
        uint32_t nL[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            // Interleaved pairs: d-1 of pair i is pair i-1, d+1 is pair i+1;
            // pair 0's low half needs lane j-1's last pair (high half), and
            // the last pair's high half needs lane j+1's first pair (low half).
            const u16x2 minus = as_u16x2(
                i == 0 ? __builtin_amdgcn_alignbit(L[NP - 1], below, 16) : L[i - 1]);
            const u16x2 plus = as_u16x2(
                i == NP - 1 ? __builtin_amdgcn_alignbit(above, L[0], 16) : L[i + 1]);
            u16x2 tt = __builtin_elementwise_min(minus, plus) + vP1;
            tt = __builtin_elementwise_min(tt, as_u16x2(L[i]));
            tt = __builtin_elementwise_min(tt, vMP2);
            tt = tt - vM + as_u16x2(c[i]);
            nL[i] = as_u32(tt);
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) L[i] = nL[i];
        if (t < len) {
            if constexpr (ATOMIC) {
                SF_BOUNDS((size_t)(stS - S) + K <= (size_t)H * W * D, CHK_SGM_SLAB);
                emit<K, true>(L, nullptr, stS);
            } else {
                SF_BOUNDS((size_t)st + K <= (size_t)H * W * D, CHK_SGM_SLAB);
                emit_buf<K>(L, rs_out, st);
            }
        }
        if constexpr (ATOMIC)
            stS += bstep;
        else
            st += (uint32_t)bstep;
        u16x2 m2 = as_u16x2(L[0]);
#pragma unroll
        for (int i = 1; i < NP; ++i) m2 = __builtin_elementwise_min(m2, as_u16x2(L[i]));
        M = row16_min(min((uint32_t)m2.x, (uint32_t)m2.y));
    };

    Raw bufA[U], bufB[U];
    uint32_t ibA[U], ibB[U];
    fetch(0, bufA, ibA);
    for (int t0 = 0; t0 < len; t0 += 2 * U) {
        fetch(t0 + U, bufB, ibB);
#pragma unroll
        for (int u = 0; u < U; ++u) step(t0 + u, bufA[u], ibA[u]);
        fetch(t0 + 2 * U, bufA, ibA);
#pragma unroll
        for (int u = 0; u < U; ++u) step(t0 + U + u, bufB[u], ibB[u]);
    }
    (void)fP2;
}

// One view; block b, row q -> chain g = 16 b + q, mapped through the table.
template <int K, bool ATOMIC, bool ADAPT>
__global__ __launch_bounds__(SGM_NT) void sgm_paths_kernel(const uint8_t *__restrict__ cost,
                                                           int H, int W, int P1, int P2,
                                                           PathTable tab, uint8_t *__restrict__ slab,
                                                           uint16_t *__restrict__ S,
                                                           const uint8_t *__restrict__ img, int pitch)
{
    constexpr int D = 16 * K;
    // The direction is uniform over the block (whole blocks per direction), so
    // the slab's buffer resource stays in scalar registers.
    const int g0 = blockIdx.x * SGM_CPB;
    int k = 0;
    while (g0 >= tab.off[k + 1]) ++k;
    const int l = g0 - tab.off[k] + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    if (l >= tab.n[k]) return;
    const size_t npx = (size_t)H * W;
    uint8_t *sl = ATOMIC ? nullptr : slab + (size_t)k * npx * D;
    sgm_chain<K, ATOMIC, SGM_U, ADAPT>(cost, sl, S, H, W, P1, P2, tab.dir[k], l, j, img, pitch);
}

// One view in census mode (CEN = 1 left base, 2 right base): no cost volume.
template <int K, bool ATOMIC, int CEN>
__global__ __launch_bounds__(SGM_NT) void sgm_paths_census_kernel(const uint64_t *__restrict__ cen_b,
                                                                  const uint64_t *__restrict__ cen_m,
                                                                  int H, int W, int P1, int P2,
                                                                  PathTable tab, uint8_t *__restrict__ slab,
                                                                  uint16_t *__restrict__ S)
{
    constexpr int D = 16 * K;
    const int g0 = blockIdx.x * SGM_CPB;  // whole blocks per direction, as sgm_paths_kernel
    int k = 0;
    while (g0 >= tab.off[k + 1]) ++k;
    const int l = g0 - tab.off[k] + (threadIdx.x >> 4);
    const int j = threadIdx.x & 15;
    if (l >= tab.n[k]) return;
    const size_t npx = (size_t)H * W;
    uint8_t *sl = ATOMIC ? nullptr : slab + (size_t)k * npx * D;
    sgm_chain<K, ATOMIC, sgm_cen_u<K>(), false, false, CEN>(nullptr, sl, S, H, W, P1, P2, tab.dir[k], l, j,
                                                            nullptr, 0, cen_b, cen_m);
}

// Many views from a task table (all tasks of one launch share K = D / 16).
// A block of 16 * c threads runs one task of up to c chains.  persistent:
// gridDim.x (<= ntasks) blocks pull task indices from *counter until the table
// is done; otherwise block b runs task b.  The counter must be 0 at the launch
// and is 0 again when the launch ends: every block pulls exactly one index >=
// ntasks, on its way out, so the block that pulls ntasks + gridDim.x - 1 makes
// the launch's last pull and resets it (no clearing launch between frames).
template <int K, int U, bool ADAPT, bool PACK = false>
__global__ __launch_bounds__(SGM_NT) void sgm_tasks_kernel(const AggView *__restrict__ views,
                                                           const AggTask *__restrict__ tasks,
                                                           int ntasks, uint8_t *base,
                                                           int *counter, AggImages ims)
{
    __shared__ int s_task;
    const int q = threadIdx.x >> 4, j = threadIdx.x & 15;
    int ti = blockIdx.x;
    for (;;) {
        if (counter) {
            if (threadIdx.x == 0) s_task = atomicAdd(counter, 1);
            __syncthreads();
            ti = __builtin_amdgcn_readfirstlane(s_task);
            __syncthreads();
        }
        if (ti >= ntasks) {
            if (counter && threadIdx.x == 0 && ti == ntasks + (int)gridDim.x - 1) atomicExch(counter, 0);
            return;
        }
        const AggTask tk = tasks[ti];
        const AggView &v = views[tk.view];
        if (q < tk.nlines) {
            const uint8_t *cost = reinterpret_cast<const uint8_t *>((uintptr_t)base + v.cost_off);
            uint8_t *slab = reinterpret_cast<uint8_t *>((uintptr_t)base + v.slab_off) +
                            (size_t)tk.slot * v.H * v.W * (16 * K);
            const uint8_t *img = ADAPT ? ims.img[tk.view] : nullptr;
            const int pitch = ADAPT ? ims.pitch[tk.view] : 0;
            sgm_chain<K, false, U, ADAPT, PACK>(cost, slab, nullptr, v.H, v.W, v.P1, v.P2, v.dir[tk.slot],
                                                tk.line0 + q, j, img, pitch);
        }
        if (!counter) return;
    }
}

// S[p][d] = sum over the n slabs; one thread per (pixel, lane chunk of K
// bytes), undoing the interleaved order of the chunk (position e <-> d = jK +
// e/2 + (e%2) K/2).
template <int K>
__global__ __launch_bounds__(256) void slab_sum_kernel(const uint8_t *__restrict__ slab, int n,
                                                       size_t npx, uint16_t *__restrict__ S)
{
    constexpr int D = 16 * K, NP = K / 2;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npx * 16) return;
    const size_t p = t >> 4;
    const int j = (int)(t & 15);
    const size_t cells = npx * D;
    const size_t off = p * D + (size_t)j * K;
    uint32_t acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = 0;
    for (int k = 0; k < n; ++k) {
        const uint8_t *src = slab + (size_t)k * cells + off;
#pragma unroll
        for (int i = 0; i < NP; ++i) acc[i] += (uint32_t)src[2 * i] | ((uint32_t)src[2 * i + 1] << 16);
    }
    uint16_t *dst = S + off;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        dst[i] = (uint16_t)(acc[i] & 0xFFFFu);
        dst[NP + i] = (uint16_t)(acc[i] >> 16);
    }
}

__global__ void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

// 0 = automatic, 1 = u8 slabs + sum, 2 = packed atomics into S.
static int g_epilogue_mode = 0;

template <int K>
static void launch_paths(bool atomic, int nblk, hipStream_t st, const uint8_t *cost, int H, int W,
                         int P1, int P2, const PathTable &tab, uint8_t *slab, uint16_t *S,
                         const uint8_t *img, int pitch)
{
    if (img) {
        if (atomic)
            hipLaunchKernelGGL((sgm_paths_kernel<K, true, true>), dim3(nblk), dim3(SGM_NT), 0, st,
                               cost, H, W, P1, P2, tab, slab, S, img, pitch);
        else
            hipLaunchKernelGGL((sgm_paths_kernel<K, false, true>), dim3(nblk), dim3(SGM_NT), 0, st,
                               cost, H, W, P1, P2, tab, slab, S, img, pitch);
    } else {
        if (atomic)
            hipLaunchKernelGGL((sgm_paths_kernel<K, true, false>), dim3(nblk), dim3(SGM_NT), 0, st,
                               cost, H, W, P1, P2, tab, slab, S, img, pitch);
        else
            hipLaunchKernelGGL((sgm_paths_kernel<K, false, false>), dim3(nblk), dim3(SGM_NT), 0, st,
                               cost, H, W, P1, P2, tab, slab, S, img, pitch);
    }
}

template <int K>
static void launch_paths_census(bool atomic, int right, int nblk, hipStream_t st, const uint64_t *cb,
                                const uint64_t *cm, int H, int W, int P1, int P2, const PathTable &tab,
                                uint8_t *slab, uint16_t *S)
{
    if (right) {
        if (atomic)
            hipLaunchKernelGGL((sgm_paths_census_kernel<K, true, 2>), dim3(nblk), dim3(SGM_NT), 0, st, cb, cm, H,
                               W, P1, P2, tab, slab, S);
        else
            hipLaunchKernelGGL((sgm_paths_census_kernel<K, false, 2>), dim3(nblk), dim3(SGM_NT), 0, st, cb, cm, H,
                               W, P1, P2, tab, slab, S);
    } else {
        if (atomic)
            hipLaunchKernelGGL((sgm_paths_census_kernel<K, true, 1>), dim3(nblk), dim3(SGM_NT), 0, st, cb, cm, H,
                               W, P1, P2, tab, slab, S);
        else
            hipLaunchKernelGGL((sgm_paths_census_kernel<K, false, 1>), dim3(nblk), dim3(SGM_NT), 0, st, cb, cm, H,
                               W, P1, P2, tab, slab, S);
    }
}

// --- task tables (host) ------------------------------------------------------

int chains_of(int r, int H, int W) { return r < 2 ? H : (r < 4 ? W : W + H - 1); }

static int chain_len(int r, int l, int H, int W)
{
    if (r < 2) return W;
    if (r < 4) return H;
    // Diagonals: lines starting on the x edge (l < H) then on the y edge.
    static const int d[8][2] = {{+1, 0}, {-1, 0}, {0, +1}, {0, -1},
                                {+1, +1}, {-1, +1}, {+1, -1}, {-1, -1}};
    const int rx = d[r][0], ry = d[r][1];
    int x, y;
    if (l < H) {
        x = rx > 0 ? 0 : W - 1;
        y = ry > 0 ? l : H - 1 - l;
    } else {
        const int k = l - H;
        x = rx > 0 ? k + 1 : W - 2 - k;
        y = ry > 0 ? 0 : H - 1;
    }
    const int nx = rx > 0 ? W - x : x + 1, ny = ry > 0 ? H - y : y + 1;
    return nx < ny ? nx : ny;
}

void append_agg_tasks(std::vector<AggTask> &tasks, std::vector<int> &task_len, int view,
                      const AggView &v, int chains_per_task)
{
    for (int s = 0; s < v.ndir; ++s) {
        const int r = v.dir[s];
        const int n = chains_of(r, v.H, v.W);
        for (int l0 = 0; l0 < n; l0 += chains_per_task) {
            AggTask t{view, s, l0, n - l0 < chains_per_task ? n - l0 : chains_per_task};
            int mx = 0;
            for (int l = l0; l < l0 + t.nlines; ++l) mx = std::max(mx, chain_len(r, l, v.H, v.W));
            tasks.push_back(t);
            task_len.push_back(mx * v.K);
        }
    }
}

void sort_tasks_longest_first(std::vector<AggTask> &tasks, const std::vector<int> &task_len)
{
    std::vector<int> idx(tasks.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return task_len[a] > task_len[b]; });
    std::vector<AggTask> out(tasks.size());
    for (size_t i = 0; i < idx.size(); ++i) out[i] = tasks[idx[i]];
    tasks.swap(out);
}

template <int K, bool PACK>
static void launch_tasks_kp(int U, int nb, int nthr, hipStream_t st, const AggView *v,
                            const AggTask *t, int n, uint8_t *base, int *counter, const AggImages &ims)
{
    if (ims.n > 0) {
        if (U == 4)
            hipLaunchKernelGGL((sgm_tasks_kernel<K, 4, true, PACK>), dim3(nb), dim3(nthr), 0, st, v, t, n,
                               base, counter, ims);
        else
            hipLaunchKernelGGL((sgm_tasks_kernel<K, 8, true, PACK>), dim3(nb), dim3(nthr), 0, st, v, t, n,
                               base, counter, ims);
    } else {
        if (U == 4)
            hipLaunchKernelGGL((sgm_tasks_kernel<K, 4, false, PACK>), dim3(nb), dim3(nthr), 0, st, v, t, n,
                               base, counter, ims);
        else
            hipLaunchKernelGGL((sgm_tasks_kernel<K, 8, false, PACK>), dim3(nb), dim3(nthr), 0, st, v, t, n,
                               base, counter, ims);
    }
}

template <int K>
static void launch_tasks_k(int U, int nb, int nthr, hipStream_t st, const AggView *v,
                           const AggTask *t, int n, uint8_t *base, int *counter, const AggImages &ims,
                           bool packed)
{
    if constexpr (K == 8 || K == 16) {
        if (packed) {
            launch_tasks_kp<K, true>(U, nb, nthr, st, v, t, n, base, counter, ims);
            return;
        }
    }
    launch_tasks_kp<K, false>(U, nb, nthr, st, v, t, n, base, counter, ims);
}

int launch_agg_tasks(const AggView *d_views, const AggTask *d_tasks, int ntasks, int K,
                     uint8_t *base, int *d_counter, int persistent_blocks, hipStream_t st,
                     int chains_per_block, int prefetch, const AggImages *images, bool packed)
{
    if (packed && K != 8 && K != 16) return fail(SF_EINVAL, "launch_agg_tasks: packed costs need D = 128 or 256");
    AggImages ims{};
    if (images) ims = *images;
    if (ims.n < 0 || ims.n > AGG_MAX_IMG) return fail(SF_EINVAL, "launch_agg_tasks: bad image count");
    for (int i = 0; i < ims.n; ++i)
        if (!ims.img[i]) return fail(SF_EINVAL, "launch_agg_tasks: NULL base image");
    if (ntasks <= 0) return SF_OK;
    if (chains_per_block != 4 && chains_per_block != 8 && chains_per_block != 16)
        return fail(SF_EINVAL, "launch_agg_tasks: chains per block must be 4, 8 or 16");
    if (prefetch != 4 && prefetch != 8) return fail(SF_EINVAL, "launch_agg_tasks: prefetch must be 4 or 8");
    int nb = ntasks;
    int *counter = nullptr;
    if (persistent_blocks > 0) {
        // *d_counter is 0 here: zeroed with the table and reset by every launch.
        nb = persistent_blocks < ntasks ? persistent_blocks : ntasks;
        counter = d_counter;
    }
    ProfScope prof("sgm_tasks", st);  // the aggregation launch alone
    const int nthr = 16 * chains_per_block;
    switch (K) {
    case 2: launch_tasks_k<2>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    case 4: launch_tasks_k<4>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    case 6: launch_tasks_k<6>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    case 8: launch_tasks_k<8>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    case 10: launch_tasks_k<10>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    case 12: launch_tasks_k<12>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    case 14: launch_tasks_k<14>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    case 16: launch_tasks_k<16>(prefetch, nb, nthr, st, d_views, d_tasks, ntasks, base, counter, ims, packed); break;
    default: return fail(SF_EUNSUPPORTED, "launch_agg_tasks: unsupported K");
    }
    const int rc = launch_status("sgm_tasks_kernel");
    if (rc && counter)  // the launch did not run: leave the counter at 0 for the next one
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t *>(counter),
                           (size_t)1, 0u);
    return rc;
}

}  // namespace sf

using namespace sf;

extern "C" int sf_sgm_set_epilogue(int mode)
{
    if (mode < 0 || mode > 2) return fail(SF_EINVAL, "sf_sgm_set_epilogue: mode must be 0, 1 or 2");
    g_epilogue_mode = mode;
    return SF_OK;
}

extern "C" size_t sf_sgm_workspace_bytes(int H, int W, int D)
{
    if (H <= 0 || W <= 0 || D <= 0) return 0;
    return (size_t)8 * H * W * D;
}

// cen_b != NULL: census mode (costs from cen_b / cen_m, base_is_right), cost unused.
static int aggregate_impl(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W, int D,
                          int P1, int P2, uint32_t path_mask, uint16_t *S, void *workspace,
                          size_t ws_bytes, void *stream, const uint64_t *cen_b = nullptr,
                          const uint64_t *cen_m = nullptr, int base_is_right = 0)
{
    SF_REQUIRE((cost || cen_b) && S, SF_EINVAL, "sf_sgm_aggregate: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_sgm_aggregate: H and W must be positive");
    SF_REQUIRE(P1 >= 0 && P2 >= P1, SF_EINVAL, "sf_sgm_aggregate: need 0 <= P1 <= P2");
    SF_REQUIRE(P2 <= 8000, SF_EINVAL, "sf_sgm_aggregate: P2 > 8000 would overflow uint16 S");
    SF_REQUIRE(path_mask >= 1 && path_mask <= 255, SF_EINVAL,
               "sf_sgm_aggregate: path_mask must be in [1, 255]");
    SF_REQUIRE(D >= 1 && D <= SF_DMAX, SF_EINVAL, "sf_sgm_aggregate: D must be in [1, 256]");
    SF_REQUIRE(D % 32 == 0, SF_EUNSUPPORTED,
               "sf_sgm_aggregate: these kernels need D to be a multiple of 32");
    SF_REQUIRE((long long)H * W <= (1LL << 28), SF_EINVAL, "sf_sgm_aggregate: image too large");
    SF_REQUIRE((long long)H * W * D <= 0x7FFFFFFFLL, SF_EINVAL,
               "sf_sgm_aggregate: H * W * D must stay below 2^31 (32-bit volume offsets)");
    PathTable tab{};
    tab.off[0] = 0;
    for (int r = 0; r < 8; ++r) {
        if (!(path_mask & (1u << r))) continue;
        tab.dir[tab.ndir] = r;
        tab.n[tab.ndir] = chains_of(r, H, W);
        tab.off[tab.ndir + 1] = tab.off[tab.ndir] + (tab.n[tab.ndir] + SGM_CPB - 1) / SGM_CPB * SGM_CPB;
        ++tab.ndir;
    }
    const size_t ncell = (size_t)H * W * D;
    bool atomic = g_epilogue_mode == 2;
    if (SF_CMAX + P2 > 255) atomic = true;  // Lr no longer fits a u8 slab
    const size_t need = atomic ? 0 : (size_t)tab.ndir * ncell;
    if (!atomic) {
        SF_REQUIRE(workspace, SF_EINVAL, "sf_sgm_aggregate: NULL workspace");
        SF_REQUIRE(ws_bytes >= need, SF_ENOMEM, "sf_sgm_aggregate: workspace too small");
    }
    hipStream_t st = as_stream(stream);
    uint8_t *slab = static_cast<uint8_t *>(workspace);
    if (atomic) {
        size_t nw = ncell / 2;  // D is even
        hipLaunchKernelGGL(fill_u32_kernel, dim3(2048), dim3(256), 0, st,
                           reinterpret_cast<uint32_t *>(S), nw, 0u);
        int rc = launch_status("fill_u32_kernel");
        if (rc) return rc;
    }
    const int nblk = tab.off[tab.ndir] / SGM_CPB;
    if (cen_b) {
        ProfScope prof("sgm_paths", st);
        switch (D / 16) {
#define SF_CEN_CASE(KK)                                                                                  \
    case KK:                                                                                             \
        launch_paths_census<KK>(atomic, base_is_right, nblk, st, cen_b, cen_m, H, W, P1, P2, tab, slab, S); \
        break;
            SF_CEN_CASE(2) SF_CEN_CASE(4) SF_CEN_CASE(6) SF_CEN_CASE(8) SF_CEN_CASE(10) SF_CEN_CASE(12)
            SF_CEN_CASE(14) SF_CEN_CASE(16)
#undef SF_CEN_CASE
        default: return fail(SF_EUNSUPPORTED, "sf_sgm_aggregate_census: unsupported D");
        }
    } else {
        ProfScope prof("sgm_paths", st);
        switch (D / 16) {
        case 2: launch_paths<2>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        case 4: launch_paths<4>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        case 6: launch_paths<6>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        case 8: launch_paths<8>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        case 10: launch_paths<10>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        case 12: launch_paths<12>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        case 14: launch_paths<14>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        case 16: launch_paths<16>(atomic, nblk, st, cost, H, W, P1, P2, tab, slab, S, img, pitch); break;
        default: return fail(SF_EUNSUPPORTED, "sf_sgm_aggregate: unsupported D");
        }
    }
    int rc = launch_status("sgm_paths_kernel");
    if (rc || atomic) return rc;
    const size_t npx = (size_t)H * W;
    const unsigned nblk_sum = (unsigned)((npx * 16 + 255) / 256);
    ProfScope prof("slab_sum", st);
    switch (D / 16) {
#define SF_SUM_CASE(KK)                                                                        \
    case KK:                                                                                   \
        hipLaunchKernelGGL(slab_sum_kernel<KK>, dim3(nblk_sum), dim3(256), 0, st, slab, tab.ndir, \
                           npx, S);                                                            \
        break;
        SF_SUM_CASE(2) SF_SUM_CASE(4) SF_SUM_CASE(6) SF_SUM_CASE(8) SF_SUM_CASE(10) SF_SUM_CASE(12)
        SF_SUM_CASE(14) SF_SUM_CASE(16)
#undef SF_SUM_CASE
    default: return fail(SF_EUNSUPPORTED, "sf_sgm_aggregate: unsupported D");
    }
    return launch_status("slab_sum_kernel");
}

extern "C" int sf_sgm_aggregate(const uint8_t *cost, int H, int W, int D, int P1, int P2,
                                uint32_t path_mask, uint16_t *S, void *workspace, size_t ws_bytes,
                                void *stream)
{
    clear_error();
    return aggregate_impl(cost, nullptr, 0, H, W, D, P1, P2, path_mask, S, workspace, ws_bytes, stream);
}

extern "C" int sf_sgm_aggregate_census(const uint64_t *cen_base, const uint64_t *cen_match, int H, int W,
                                       int D, int base_is_right, int P1, int P2, uint32_t path_mask,
                                       uint16_t *S, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(cen_base && cen_match, SF_EINVAL, "sf_sgm_aggregate_census: NULL census");
    SF_REQUIRE(base_is_right == 0 || base_is_right == 1, SF_EINVAL,
               "sf_sgm_aggregate_census: base_is_right must be 0 or 1");
    return aggregate_impl(nullptr, nullptr, 0, H, W, D, P1, P2, path_mask, S, workspace, ws_bytes, stream,
                          cen_base, cen_match, base_is_right);
}

extern "C" int sf_sgm_aggregate_adaptive(const uint8_t *cost, const uint8_t *img, int pitch, int H,
                                         int W, int D, int P1, int P2, uint32_t path_mask,
                                         uint16_t *S, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(img, SF_EINVAL, "sf_sgm_aggregate_adaptive: NULL image");
    SF_REQUIRE(pitch >= W, SF_EINVAL, "sf_sgm_aggregate_adaptive: pitch < W");
    SF_REQUIRE((long long)H * pitch <= 0x7FFFFFFFLL, SF_EINVAL, "sf_sgm_aggregate_adaptive: image too large");
    return aggregate_impl(cost, img, pitch, H, W, D, P1, P2, path_mask, S, workspace, ws_bytes, stream);
}
