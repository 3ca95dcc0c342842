// Flat parameter layout of the learned LR-check network and the per-lane
// MFMA weight fragments its fused inference kernel reads (packed once per
// inference from the FP32 parameters, by a launch of its own or as an extra
// job of the frame's census launch).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sf {

// Flat FP32 parameters (5377): W1[16][4][3][3] b1[16] W2[16][16][3][3] b2[16]
// W3[16][16][3][3] b3[16] W4[1][16][3][3] b4[1].
constexpr int LR_NP = 5377;
constexpr int OFF_W1 = 0, OFF_B1 = 576, OFF_W2 = 592, OFF_B2 = 2896, OFF_W3 = 2912, OFF_B3 = 5216,
              OFF_W4 = 5232, OFF_B4 = 5376;

// Fragment slots (uint4 per lane, 64 lanes a slot) and the biases after them.
constexpr int FP_L1 = 0, FP_L2 = 2, FP_L3 = 7, FP_L4 = 12, FP_NSLOT = 13;
constexpr int FP_FRAGS = FP_NSLOT * 64;
constexpr int FP_B1 = 0, FP_B2 = 16, FP_B3 = 32, FP_B4 = 48, FP_FLOATS = 49;

// Taps (row-major over the 3x3 window) that K = 32 MFMA q (0..3) of a
// 16-channel layer pairs, hi = 0 / 1: (0, 1), (3, 4), (6, 7), (2, 5); tap 8
// goes with zeros in MFMA 4.  Each pair is two pixels a constant distance
// apart, so one two-address LDS read fetches both channel blocks into
// consecutive registers, the order the MFMA operand needs.
__host__ __device__ constexpr int fused_tap(int q, int hi)
{
    return q == 3 ? (hi ? 5 : 2) : 3 * q + hi;
}

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u | ((u & 0x7fffffu) ? 0x400000u : 0u)) >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Lane `lane` (0..63) of fragment slot `slot` (0..FP_NSLOT-1): eight BF16
// weights in the MFMA A-operand order of the fused kernel (lane group kg =
// lane / 16 holds K elements 8 kg .. 8 kg + 7 of row n = lane % 16).  Slot 0,
// lanes < FP_FLOATS, also copy the biases.
__device__ __forceinline__ void lrnet_pack_lane(const float *__restrict__ prm, uint4 *__restrict__ frag,
                                                float *__restrict__ fl, int slot, int lane)
{
    const int n = lane & 15, kg = lane >> 4;
    // Parameter index of each of the lane's 8 values (-1: zero), all computed
    // before any load so that the 8 loads are in flight together.
    int idx[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = j & 3, hi = j >> 2;
        int k = -1;
        if (slot == FP_L1) {  // layer 1, taps kg and kg + 4, input channel i
            k = OFF_W1 + (n * 4 + i) * 9 + kg + 4 * hi;
        } else if (slot == FP_L1 + 1) {  // layer 1, tap 8 (lane group 0 only)
            if (kg == 0 && !hi) k = OFF_W1 + (n * 4 + i) * 9 + 8;
        } else if (slot < FP_L4) {  // layers 2, 3: taps fused_tap(q, 0 / 1) (q < 4) or tap 8, channel 4 kg + i
            const int q = (slot - FP_L2) % 5;
            const int off = slot < FP_L3 ? OFF_W2 : OFF_W3;
            if (q < 4) k = off + (n * 16 + 4 * kg + i) * 9 + fused_tap(q, hi);
            else if (!hi) k = off + (n * 16 + 4 * kg + i) * 9 + 8;
        } else if (n < 9 && !hi) {  // layer 4: row n = tap n, input channel 4 kg + i
            k = OFF_W4 + (4 * kg + i) * 9 + n;
        }
        idx[j] = k;
    }
    float w[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j] = prm[idx[j] < 0 ? 0 : idx[j]];
    uint16_t h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = bf16_bits(idx[j] < 0 ? 0.0f : w[j]);
    frag[slot * 64 + lane] = make_uint4((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16),
                                        (uint32_t)h[4] | ((uint32_t)h[5] << 16), (uint32_t)h[6] | ((uint32_t)h[7] << 16));
    if (slot == 0 && lane < FP_FLOATS)
        fl[lane] = prm[lane < 16 ? OFF_B1 + lane : lane < 32 ? OFF_B2 + lane - 16 : lane < 48 ? OFF_B3 + lane - 32 : OFF_B4];
}

}  // namespace sf
