// Learned stand-in for the left-right consistency check.  The check itself is
// the paper's (Sec. 3.1: comparing two computed disparity maps removes the
// inconsistent pixels); this network predicts its outcome from the left view
// alone so that the right-view aggregation can be skipped, and is trained on
// labels produced by the check.
//
// Network: 3x3 convolutions (cross-correlation, zero padding), channels
// 4 -> 16 -> 16 -> 16 -> 1, ReLU after the first three, logit output.  Layer
// inputs and weights are BF16 (round to nearest even), biases FP32, sums FP32.
// Flat FP32 parameter vector (5377): W1[16][4][3][3] b1[16] W2[16][16][3][3]
// b2[16] W3[16][16][3][3] b3[16] W4[1][16][3][3] b4[1].
//
// Inference is one fused kernel per output tile with the activations in LDS
// (lrnet_fused_kernel, all four layers on MFMA; see "fused inference" below).
// Training keeps the activations in HBM as BF16 NHWC ([B][H][W][16], 32 bytes
// per pixel) and runs the kernels:
//   l1_fwd     4 -> 16 (VALU: K = 36 is too thin for a matrix tile)
//   conv16     16 -> 16 on MFMA v_mfma_f32_16x16x16_bf16: forward (bias,
//              ReLU, BF16) or backward-data (transposed, flipped weights; the
//              ReLU mask of the layer below; BF16)
//   l4_fwd     16 -> 1 (VALU) + loss and dL/dz4 for training
//   l4_bwd     dL/dz4 -> dL/dz3 (VALU) and the W4 / b4 partial gradients
//   wgrad      dW[co][ci][tap] = sum_p gz[co](p) a[ci](p + tap - 1) on MFMA
//              (K = pixels), per-block partials reduced in a fixed order
//   adam       FP32 Adam step.
#include <mutex>

#include "lrnet_pack.hpp"
#include "sf_internal.hpp"
#include "stages.hpp"

namespace sf {


typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// The same rounding for a value that is not NaN (a ReLU output): no branch;
// exact for every other input, infinities included.
__device__ __forceinline__ uint16_t bf16_bits_nonnan(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bf16_round(float f) { return bf16_val(bf16_bits(f)); }

// --- layer 1: features (FP32, rounded to BF16 on load) -> a1 ------------------
constexpr int T1 = 16;  // 16 x 16 output pixels per block

__global__ __launch_bounds__(256) void l1_fwd_kernel(const float *__restrict__ prm,
                                                     const float4 *__restrict__ feat, int H, int W,
                                                     uint16_t *__restrict__ a1)
{
    __shared__ float s_in[T1 + 2][T1 + 2][4];
    __shared__ float s_w[16][4][9];
    __shared__ float s_b[16];
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * T1, y0 = blockIdx.y * T1;
    const int tid = threadIdx.x;
    for (int i = tid; i < 576; i += 256) (&s_w[0][0][0])[i] = bf16_round(prm[OFF_W1 + i]);
    if (tid < 16) s_b[tid] = prm[OFF_B1 + tid];
    const size_t img = (size_t)b * H * W;
    for (int i = tid; i < (T1 + 2) * (T1 + 2); i += 256) {
        int ly = i / (T1 + 2), lx = i - ly * (T1 + 2);
        int gy = y0 + ly - 1, gx = x0 + lx - 1;
        float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) f = feat[img + (size_t)gy * W + gx];
        s_in[ly][lx][0] = bf16_round(f.x);
        s_in[ly][lx][1] = bf16_round(f.y);
        s_in[ly][lx][2] = bf16_round(f.z);
        s_in[ly][lx][3] = bf16_round(f.w);
    }
    __syncthreads();
    const int tx = tid & 15, ty = tid >> 4;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= W || y >= H) return;
    uint32_t packed[8];
#pragma unroll
    for (int co = 0; co < 16; co += 2) {
        float z[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float acc = 0.0f;
#pragma unroll
            for (int ci = 0; ci < 4; ++ci)
#pragma unroll
                for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx)
                        acc = __builtin_fmaf(s_w[co + h][ci][ky * 3 + kx], s_in[ty + ky][tx + kx][ci], acc);
            acc += s_b[co + h];
            z[h] = acc > 0.0f ? acc : 0.0f;
        }
        packed[co / 2] = (uint32_t)bf16_bits(z[0]) | ((uint32_t)bf16_bits(z[1]) << 16);
    }
    uint4 *o = reinterpret_cast<uint4 *>(a1 + (img + (size_t)y * W + x) * 16);
    o[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
    o[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
}

// --- 16 -> 16 convolution on MFMA ---------------------------------------------
// Output tile 8 x 32 pixels = 16 groups of 16 consecutive pixels of a row; wave
// w computes groups w, w+4, w+8, w+12.  For each group and tap one
// v_mfma_f32_16x16x16_bf16 with
//   A[m][k] = in[pixel m shifted by the tap][channel k]   (lane: m = l%16, k = 4(l/16)+i)
//   B[k][n] = weight[tap][in channel k][out channel n]     (lane: n = l%16, k = 4(l/16)+i)
//   D[m][n] accumulates in FP32                             (lane: n = l%16, m = 4(l/16)+i)
constexpr int CT_H = 8, CT_W = 32;

template <bool BWD>
__global__ __launch_bounds__(256) void conv16_mfma_kernel(const float *__restrict__ prm, int w_off,
                                                          int b_off, const uint16_t *__restrict__ in,
                                                          const uint16_t *__restrict__ relu_src,
                                                          int H, int W, uint16_t *__restrict__ out)
{
    __shared__ __align__(16) uint16_t s_in[CT_H + 2][CT_W + 2][16];
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * CT_W, y0 = blockIdx.y * CT_H;
    const int tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    // Stage the input tile with its 1-pixel halo (zeros outside the image).
    for (int i = tid; i < (CT_H + 2) * (CT_W + 2) * 2; i += 256) {
        const int px = i >> 1, half = i & 1;
        const int ly = px / (CT_W + 2), lx = px - ly * (CT_W + 2);
        const int gy = y0 + ly - 1, gx = x0 + lx - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = reinterpret_cast<const uint4 *>(in + (img + (size_t)gy * W + gx) * 16)[half];
        reinterpret_cast<uint4 *>(&s_in[ly][lx][0])[half] = v;
    }
    const int lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, kg = lane >> 4;
    // B fragments of the 9 taps.  Forward: B[k][n] = W[n][k][ky][kx].
    // Backward-data: B[k][n] = W[k][n][2-ky][2-kx] (transpose and flip).
    bf16x4 bw[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ky = t / 3, kx = t % 3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * kg + i;
            const int idx = BWD ? ((k * 16 + n) * 9 + (2 - ky) * 3 + (2 - kx)) : ((n * 16 + k) * 9 + t);
            bw[t][i] = (short)bf16_bits(prm[w_off + idx]);
        }
    }
    const float bias = BWD ? 0.0f : prm[b_off + n];
    __syncthreads();
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        const int g = wave + 4 * gi;
        const int ty = g >> 1, tx0 = (g & 1) * 16;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ky = t / 3, kx = t % 3;
            const bf16x4 a = *reinterpret_cast<const bf16x4 *>(&s_in[ty + ky][tx0 + n + kx][4 * kg]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[t], acc, 0, 0, 0);
        }
        const int y = y0 + ty;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + tx0 + 4 * kg + i;
            if (y >= H || x >= W) continue;
            const size_t o = (img + (size_t)y * W + x) * 16 + n;
            float v;
            if (BWD) {
                // Gradient w.r.t. the pre-activation of the layer below: pass only
                // where its ReLU was active, then round to BF16.
                v = bf16_val(relu_src[o]) > 0.0f ? acc[i] : 0.0f;
            } else {
                v = acc[i] + bias;
                v = v > 0.0f ? v : 0.0f;
            }
            out[o] = bf16_bits(v);
        }
    }
}

// --- layer 4: 16 -> 1 ---------------------------------------------------------
// One thread per pixel of a 16 x 16 tile.  Inference writes the logit; training
// also writes g4 = (sigmoid(z) - y) / N and per-block partial losses.
__global__ __launch_bounds__(256) void l4_fwd_kernel(const float *__restrict__ prm,
                                                     const uint16_t *__restrict__ a3, int H, int W,
                                                     float *__restrict__ logits,
                                                     const uint8_t *__restrict__ label, float inv_n,
                                                     float *__restrict__ g4,
                                                     float *__restrict__ loss_part)
{
    __shared__ __align__(16) uint16_t s_in[T1 + 2][T1 + 2][16];
    __shared__ float s_w[16][9];
    __shared__ float s_red[256];
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * T1, y0 = blockIdx.y * T1;
    const int tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    for (int i = tid; i < 144; i += 256) (&s_w[0][0])[i] = bf16_round(prm[OFF_W4 + i]);
    for (int i = tid; i < (T1 + 2) * (T1 + 2) * 2; i += 256) {
        const int px = i >> 1, half = i & 1;
        const int ly = px / (T1 + 2), lx = px - ly * (T1 + 2);
        const int gy = y0 + ly - 1, gx = x0 + lx - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = reinterpret_cast<const uint4 *>(a3 + (img + (size_t)gy * W + gx) * 16)[half];
        reinterpret_cast<uint4 *>(&s_in[ly][lx][0])[half] = v;
    }
    __syncthreads();
    const int tx = tid & 15, ty = tid >> 4;
    const int x = x0 + tx, y = y0 + ty;
    float l = 0.0f;
    if (x < W && y < H) {
        float acc = 0.0f;
#pragma unroll
        for (int ci = 0; ci < 16; ++ci)
#pragma unroll
            for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx)
                    acc = __builtin_fmaf(s_w[ci][ky * 3 + kx], bf16_val(s_in[ty + ky][tx + kx][ci]), acc);
        const float z = acc + prm[OFF_B4];
        const size_t p = img + (size_t)y * W + x;
        if (logits) logits[p] = z;
        if (label) {
            const float yv = label[p] ? 1.0f : 0.0f;
            const float s = 1.0f / (1.0f + expf(-z));
            g4[p] = (s - yv) * inv_n;
            const float sp = z > 0.0f ? z + log1pf(expf(-z)) : log1pf(expf(z));
            l = sp - yv * z;
        }
    }
    if (loss_part) {
        s_red[tid] = l;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) s_red[tid] += s_red[tid + s];
            __syncthreads();
        }
        if (tid == 0)
            loss_part[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s_red[0];
    }
}

// dL/dz3[q][ci] = bf16( sum_tap W4[ci][tap] g4(q - tap + 1) * [a3(q, ci) > 0] ), and the
// W4 / b4 partial gradients sum_p g4(p) a3[ci](p + tap - 1), sum_p g4(p) of this tile.
__global__ __launch_bounds__(256) void l4_bwd_kernel(const float *__restrict__ prm,
                                                     const float *__restrict__ g4,
                                                     const uint16_t *__restrict__ a3, int H, int W,
                                                     uint16_t *__restrict__ gz3,
                                                     float *__restrict__ part)
{
    __shared__ float s_g[T1 + 2][T1 + 2];
    __shared__ __align__(16) uint16_t s_a[T1 + 2][T1 + 2][16];
    __shared__ float s_w[16][9];
    __shared__ float s_red[145][8];
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * T1, y0 = blockIdx.y * T1;
    const int tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    for (int i = tid; i < 144; i += 256) (&s_w[0][0])[i] = bf16_round(prm[OFF_W4 + i]);
    for (int i = tid; i < (T1 + 2) * (T1 + 2); i += 256) {
        const int ly = i / (T1 + 2), lx = i - ly * (T1 + 2);
        const int gy = y0 + ly - 1, gx = x0 + lx - 1;
        const bool in_img = gy >= 0 && gy < H && gx >= 0 && gx < W;
        s_g[ly][lx] = in_img ? g4[img + (size_t)gy * W + gx] : 0.0f;
        const uint4 *src = reinterpret_cast<const uint4 *>(a3 + (img + (size_t)gy * W + gx) * 16);
        uint4 v0 = make_uint4(0u, 0u, 0u, 0u), v1 = v0;
        if (in_img) { v0 = src[0]; v1 = src[1]; }
        reinterpret_cast<uint4 *>(&s_a[ly][lx][0])[0] = v0;
        reinterpret_cast<uint4 *>(&s_a[ly][lx][0])[1] = v1;
    }
    __syncthreads();
    const int tx = tid & 15, ty = tid >> 4;
    const int x = x0 + tx, y = y0 + ty;
    const bool inside = x < W && y < H;
    if (inside) {
        uint32_t packed[8];
#pragma unroll
        for (int ci = 0; ci < 16; ci += 2) {
            float v[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float acc = 0.0f;
#pragma unroll
                for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx)
                        acc = __builtin_fmaf(s_w[ci + h][ky * 3 + kx], s_g[ty + 2 - ky][tx + 2 - kx], acc);
                v[h] = bf16_val(s_a[ty + 1][tx + 1][ci + h]) > 0.0f ? acc : 0.0f;
            }
            packed[ci / 2] = (uint32_t)bf16_bits(v[0]) | ((uint32_t)bf16_bits(v[1]) << 16);
        }
        uint4 *o = reinterpret_cast<uint4 *>(gz3 + (img + (size_t)y * W + x) * 16);
        o[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
        o[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
    }
    // Partial weight gradients: thread handles parameter i = tid (< 145), summing
    // over the tile's 256 pixels in a fixed order.
    if (tid < 145) {
        float acc = 0.0f;
        if (tid < 144) {
            const int ci = tid / 9, t = tid % 9, ky = t / 3, kx = t % 3;
            for (int p = 0; p < 256; ++p) {
                const int py = p >> 4, pxl = p & 15;
                acc = __builtin_fmaf(s_g[py + 1][pxl + 1], bf16_val(s_a[py + ky][pxl + kx][ci]), acc);
            }
        } else {
            for (int p = 0; p < 256; ++p) acc += s_g[(p >> 4) + 1][(p & 15) + 1];
        }
        const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[blk * 145 + tid] = acc;
    }
}

// --- weight gradients of a 16-output layer on MFMA ------------------------------
// dW[co][ci][tap] = sum_p gz[co](p) a[ci](p + tap - 1), db[co] = sum_p gz[co](p)
// over a tile of 8 x 32 pixels; CIN = 16 (a = BF16 NHWC16 activations) or 4
// (a = FP32 features, rounded to BF16, padded to 16 channels with zeros).
// MFMA: M = co, N = ci, K = 16 pixels of one tile row half; each wave takes 4 of
// the 16 pixel groups and all 9 taps; the 4 waves' sums are added in order.
template <int CIN>
__global__ __launch_bounds__(256) void wgrad_mfma_kernel(const uint16_t *__restrict__ gz,
                                                         const uint16_t *__restrict__ a16,
                                                         const float4 *__restrict__ a4, int H,
                                                         int W, float *__restrict__ part)
{
    constexpr int NPART = 16 * CIN * 9 + 16;
    __shared__ __align__(16) uint16_t s_a[CT_H + 2][CT_W + 2][16];
    __shared__ __align__(16) uint16_t s_g[CT_H][CT_W][16];
    __shared__ float s_acc[4][9][4][64];
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * CT_W, y0 = blockIdx.y * CT_H;
    const int tid = threadIdx.x;
    const size_t img = (size_t)b * H * W;
    for (int i = tid; i < (CT_H + 2) * (CT_W + 2) * 2; i += 256) {
        const int px = i >> 1, half = i & 1;
        const int ly = px / (CT_W + 2), lx = px - ly * (CT_W + 2);
        const int gy = y0 + ly - 1, gx = x0 + lx - 1;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            if (CIN == 16) {
                v = reinterpret_cast<const uint4 *>(a16 + (img + (size_t)gy * W + gx) * 16)[half];
            } else if (half == 0) {
                const float4 f = a4[img + (size_t)gy * W + gx];
                v.x = (uint32_t)bf16_bits(f.x) | ((uint32_t)bf16_bits(f.y) << 16);
                v.y = (uint32_t)bf16_bits(f.z) | ((uint32_t)bf16_bits(f.w) << 16);
            }
        }
        reinterpret_cast<uint4 *>(&s_a[ly][lx][0])[half] = v;
    }
    for (int i = tid; i < CT_H * CT_W * 2; i += 256) {
        const int px = i >> 1, half = i & 1;
        const int ly = px / CT_W, lx = px - ly * CT_W;
        const int gy = y0 + ly, gx = x0 + lx;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gy < H && gx < W) v = reinterpret_cast<const uint4 *>(gz + (img + (size_t)gy * W + gx) * 16)[half];
        reinterpret_cast<uint4 *>(&s_g[ly][lx][0])[half] = v;
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int mn = lane & 15, kg = lane >> 4;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.0f;
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
        const int g = wave + 4 * gi;
        const int ty = g >> 1, tx0 = (g & 1) * 16;
        // A[m = co][k = pixel]: lane holds co = mn, pixels 4 kg + i of the group.
        bf16x4 av;
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = (short)s_g[ty][tx0 + 4 * kg + i][mn];
#pragma unroll
        for (int i = 0; i < 4; ++i) dbias += bf16_val((uint16_t)av[i]);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ky = t / 3, kx = t % 3;
            // B[k = pixel][n = ci]: lane holds ci = mn, pixels 4 kg + i, shifted by the tap.
            bf16x4 bv;
#pragma unroll
            for (int i = 0; i < 4; ++i) bv[i] = (short)s_a[ty + ky][tx0 + 4 * kg + i + kx][mn];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[t], 0, 0, 0);
        }
    }
    // D[m = co][n = ci]: lane holds ci = mn, co = 4 kg + i.
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) s_acc[wave][t][i][lane] = acc[t][i];
    __syncthreads();
    const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float *pp = part + blk * NPART;
    for (int e = tid; e < 16 * CIN * 9; e += 256) {
        const int co = e / (CIN * 9), rem = e - co * CIN * 9, ci = rem / 9, t = rem % 9;
        const int i = co & 3, kgo = co >> 2;
        const int l = kgo * 16 + ci;
        pp[e] = ((s_acc[0][t][i][l] + s_acc[1][t][i][l]) + s_acc[2][t][i][l]) + s_acc[3][t][i][l];
    }
    // Bias: lanes with the same co (= mn) across kg and waves.
    __syncthreads();
    float *s_db = &s_acc[0][0][0][0];
    s_db[tid] = dbias;  // tid = wave * 64 + kg * 16 + co
    __syncthreads();
    if (tid < 16) {
        float s = 0.0f;
        for (int w = 0; w < 4; ++w)
            for (int k = 0; k < 4; ++k) s += s_db[w * 64 + k * 16 + tid];
        pp[16 * CIN * 9 + tid] = s;
    }
}

// Sum over blocks, in block order, of the partial gradients part[blk][e]; slot
// e < nw is weight woff + e, the rest biases boff + (e - nw).
__global__ void reduce_parts_kernel(const float *__restrict__ part, int nblk, int npart, int nw,
                                    int woff, int boff, float *__restrict__ grad)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npart) return;
    float s = 0.0f;
    for (int bk = 0; bk < nblk; ++bk) s += part[(size_t)bk * npart + e];
    grad[e < nw ? woff + e : boff + (e - nw)] = s;
}

__global__ void sum_kernel(const float *__restrict__ v, int n, float scale, float *__restrict__ out)
{
    __shared__ float s[256];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0] * scale;
}

__global__ void adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int n, float lr, float b1, float b2,
                            float eps, float b1t, float b2t)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - b1t);
    const float vh = vi / (1.0f - b2t);
    w[i] = w[i] - (lr * mh) / (sqrtf(vh) + eps);
}

// Learned mask: valid iff the logit is positive and x - d* >= 0 (a match pixel
// outside the image can never pass the check); disp = d_sub where valid, else -1.
__global__ void lr_mask_kernel(const float *__restrict__ logits, const int16_t *__restrict__ wta,
                               const float *__restrict__ dsub, int H, int W,
                               uint8_t *__restrict__ valid, float *__restrict__ disp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= H * W) return;
    const int x = i % W;
    const int ok = logits[i] > 0.0f && x - (int)wta[i] >= 0;
    valid[i] = (uint8_t)ok;
    disp[i] = ok ? dsub[i] : -1.0f;
}


// --- fused inference: all four layers per tile, activations in LDS --------------
// Output tile FT_H x FT_W; the layer inputs are kept on halos shrinking by one
// pixel per layer (features 24 x 40, a1 22 x 38, a2 20 x 36, a3 18 x 34).  Pixels
// of a halo that fall outside the image hold 0 (zero padding of every layer).
// All four layers run on MFMA over groups of 16 consecutive pixels of a region
// (row-major).  The weights are the A operand (rows = output channels) and the
// activations the B operand (columns = pixels), so each lane ends up holding
// four consecutive output channels of one pixel.  Its accumulator starts at
// the four biases; the epilogue applies ReLU and zero padding, rounds to BF16
// (v_cvt_pk_bf16_f32, round to nearest even) and stores the four channels with
// one 8-byte LDS write.  A 3x3 layer with 16 input channels takes five
// v_mfma_f32_16x16x32_bf16: lane group kg contributes channels 4kg..4kg+3 of
// the taps (0,1), (2,3), (4,5), (6,7), then of tap 8 with a zero upper half.
// Layer 1 (4 channels) takes two: taps kg and kg + 4, then tap 8 (group 0).
// The contraction pairs the elements of A and B by lane group and position, so
// any consistent assignment of (tap, channel) to positions gives the same sum
// of products, and one chain uses one MFMA opcode.  Layer 4 (one output
// channel) puts its 9 taps on the rows of A: one MFMA per 16 pixels gives the
// per-tap channel sums P_t(p), which go to LDS, and the logit at p is
// b4 + sum over taps t of P_t(p + offset_t).  Weight fragments come pre-packed
// per lane (lrnet_pack_lane: pack_fused_kernel, or the learned frame's census
// launch), 16 bytes per lane and slot; each block copies them to LDS while its
// features load.
constexpr int FT_H = 16, FT_W = 32;
constexpr int FT_NW = 16;  // waves per block: they share the tile's LDS, so more of them hide latency

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two FP32 values -> packed BF16 (low half = a), round to nearest even (a NaN
// stays a NaN).
__device__ __forceinline__ uint32_t bf16x2_bits(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2v));
}

// Pixel offset of tap t (row-major over the 3x3 window) in a region of width wi.
__device__ __forceinline__ int tap_off(int t, int wi) { return (t / 3) * wi + t % 3; }

__global__ void pack_fused_kernel(const float *__restrict__ prm, uint4 *__restrict__ frag,
                                  float *__restrict__ fl)
{
    lrnet_pack_lane(prm, frag, fl, blockIdx.x, threadIdx.x & 63);
}

// Pixels per plane of a 16-channel activation array of np pixels: the least
// count >= np that is 16 mod 32, so that planes start 128 bytes apart modulo
// the 256 bytes that the LDS banks span.
__host__ __device__ constexpr int plane_px(int np) { return ((np + 15) & ~31) + 16; }

// Offset (in BF16 elements) of channels 4 kg .. 4 kg + 3 of pixel p in a
// 16-channel activation array of np pixels, stored as four planes of channel
// blocks (plane kg holds channels 4 kg .. 4 kg + 3 of every pixel, 8 bytes per
// pixel).  The 8-byte accesses of one channel block by 16 consecutive pixels
// are 128 contiguous bytes, two lane groups on neighbouring planes fall on
// disjoint banks (plane_px), and the nine taps of a 3x3 window are constant
// offsets from one base address.
__device__ __forceinline__ int act_off(int p, int kg, int np) { return (kg * plane_px(np) + p) * 4; }

// ReLU with the maxNum rule: x for x > 0, else 0, and 0 for a NaN.
__device__ __forceinline__ float relu_mfma(float x) { return __builtin_fmaxf(x, 0.0f); }

__device__ __forceinline__ bf16x8 join8(uint2 lo, uint2 hi)
{
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

// One 3x3 MFMA layer over a region: input sIn [hi][wi][C] (bf16; C = 16 arrays
// in channel-block planes, act_off), output sOut [hi-2][wi-2][16] (planes); (gy0, gx0) =
// image coordinates of the output region's first pixel; bias = the biases of
// output channels 4 kg .. 4 kg + 3; frag = the layer's first weight slot.
template <int C>
__device__ __forceinline__ void fused_layer(const uint16_t *sIn, int hi, int wi, uint16_t *sOut,
                                            const uint4 *__restrict__ frag, f32x4 bias, int gy0,
                                            int gx0, int H, int W, int lane, int wave)
{
    constexpr int NQ = C == 16 ? 5 : 2;  // K = 32 MFMAs; the last one holds tap 8 and zeros
    const int ho = hi - 2, wo = wi - 2, nout = ho * wo;
    const int n = lane & 15, kg = lane >> 4;
    bf16x8 w32[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) w32[q] = __builtin_bit_cast(bf16x8, frag[q * 64 + lane]);
    // Zero padding is needed only where the output region reaches outside the image.
    const bool interior = gy0 >= 0 && gx0 >= 0 && gy0 + ho <= H && gx0 + wo <= W;
    const int ngroups = (nout + 15) >> 4;
    const uint2 zero2 = make_uint2(0u, 0u);
    for (int g = wave; g < ngroups; g += FT_NW) {
        const int mo = g * 16 + n;
        const int m = mo < nout ? mo : nout - 1;
        const int oy = m / wo, ox = m - oy * wo;
        const int p0 = oy * wi + ox;
        // All LDS reads of the group are issued before the MFMA chain uses any.
        bf16x8 b32[NQ];
        if (C == 16) {
            const uint16_t *base = sIn + act_off(p0, kg, hi * wi);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                b32[q] = join8(*reinterpret_cast<const uint2 *>(base + 4 * tap_off(fused_tap(q, 0), wi)),
                               *reinterpret_cast<const uint2 *>(base + 4 * tap_off(fused_tap(q, 1), wi)));
            b32[4] = join8(*reinterpret_cast<const uint2 *>(base + 4 * tap_off(8, wi)), zero2);
        } else {
            b32[0] = join8(*reinterpret_cast<const uint2 *>(sIn + (p0 + tap_off(kg, wi)) * 4),
                           *reinterpret_cast<const uint2 *>(sIn + (p0 + tap_off(kg + 4, wi)) * 4));
            uint2 t8 = zero2;
            if (kg == 0) t8 = *reinterpret_cast<const uint2 *>(sIn + (p0 + tap_off(8, wi)) * 4);
            b32[1] = join8(t8, zero2);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the chain
        f32x4 acc = bias;
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w32[q], b32[q], acc, 0, 0, 0);
        if (mo >= nout) continue;
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = relu_mfma(acc[i]);
        if (!interior) {  // uniform over the block
            const int gy = gy0 + oy, gx = gx0 + ox;
            if (!((unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W)) {
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = 0.0f;  // zero padding outside the image
            }
        }
        *reinterpret_cast<uint2 *>(sOut + act_off(mo, kg, nout)) = make_uint2(bf16x2_bits(v[0], v[1]), bf16x2_bits(v[2], v[3]));
    }
}

__global__ __launch_bounds__(64 * FT_NW) __attribute__((amdgpu_waves_per_eu(8, 8))) void lrnet_fused_kernel(const uint4 *__restrict__ frag,
                                                                 const float *__restrict__ fl,
                                                                 const float4 *__restrict__ feat,
                                                                 int H, int W, float *__restrict__ logits,
                                                                 LrMaskOut mask)
{
    constexpr int FH = FT_H + 8, FW = FT_W + 8;   // features
    constexpr int H1 = FT_H + 6, W1 = FT_W + 6;   // a1
    constexpr int H2 = FT_H + 4, W2 = FT_W + 4;   // a2
    constexpr int H3 = FT_H + 2, W3 = FT_W + 2;   // a3 (aliases a1)
    constexpr int N3 = H3 * W3;                   // a3 pixels; P (9 x N3 FP32) aliases a2
    static_assert(9 * N3 * 4 <= plane_px(H2 * W2) * 16 * 2, "tap sums must fit the a2 buffer");
    __shared__ __align__(16) uint16_t sF[FH * FW * 4];
    constexpr int NA1 = plane_px(H1 * W1) > plane_px(N3) ? plane_px(H1 * W1) : plane_px(N3);
    __shared__ __align__(16) uint16_t sA1[NA1 * 16];           // a1, then a3
    __shared__ __align__(16) uint16_t sA2[plane_px(H2 * W2) * 16];
    __shared__ __align__(16) uint4 sW[FP_FRAGS];  // weight fragments [slot][lane], staged from global
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * FT_W, y0 = blockIdx.y * FT_H;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t img = (size_t)b * H * W;
    for (int i = tid; i < FH * FW; i += 64 * FT_NW) {
        const int ly = i / FW, lx = i - ly * FW;
        const int gy = y0 + ly - 4, gx = x0 + lx - 4;
        float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) f = feat[img + (size_t)gy * W + gx];
        // BF16 rounding (round to nearest even; NaN stays NaN).
        reinterpret_cast<uint2 *>(sF)[i] = make_uint2(bf16x2_bits(f.x, f.y), bf16x2_bits(f.z, f.w));
    }
    for (int i = tid; i < FP_FRAGS; i += 64 * FT_NW) sW[i] = frag[i];
    __syncthreads();
    const int n = lane & 15, kg = lane >> 4;
    auto bias4 = [&](int off) { return f32x4{fl[off + 4 * kg], fl[off + 4 * kg + 1], fl[off + 4 * kg + 2], fl[off + 4 * kg + 3]}; };
    fused_layer<4>(sF, FH, FW, sA1, sW + FP_L1 * 64, bias4(FP_B1), y0 - 3, x0 - 3, H, W, lane, wave);
    __syncthreads();
    fused_layer<16>(sA1, H1, W1, sA2, sW + FP_L2 * 64, bias4(FP_B2), y0 - 2, x0 - 2, H, W, lane, wave);
    __syncthreads();
    fused_layer<16>(sA2, H2, W2, sA1, sW + FP_L3 * 64, bias4(FP_B3), y0 - 1, x0 - 1, H, W, lane, wave);
    __syncthreads();
    // Layer 4, step 1: P[t][p] = sum over the 16 channels of W4[c][t] a3[p][c], tap-major in a2's buffer.
    float *P = reinterpret_cast<float *>(sA2);
    const uint4 f4 = sW[FP_L4 * 64 + lane];
    const bf16x4 w4 = __builtin_bit_cast(bf16x4, make_uint2(f4.x, f4.y));
    for (int g = wave; g < (N3 + 15) / 16; g += FT_NW) {
        const int p = g * 16 + n;
        const int pc = p < N3 ? p : N3 - 1;
        const bf16x4 a = *reinterpret_cast<const bf16x4 *>(sA1 + act_off(pc, kg, N3));
        const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w4, a, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        if (p < N3) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (4 * kg + i < 9) P[(4 * kg + i) * N3 + p] = acc[i];
        }
    }
    __syncthreads();
    // Step 2: the logit sums the nine tap sums in tap order, then adds the bias.
    const float b4 = fl[FP_B4];
    for (int q = tid; q < FT_H * FT_W; q += 64 * FT_NW) {
        const int oy = q / FT_W, ox = q - oy * FT_W;
        const int gy = y0 + oy, gx = x0 + ox;
        if (gy >= H || gx >= W) continue;
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) s += P[t * N3 + (oy + t / 3) * W3 + ox + t % 3];
        const float logit = s + b4;
        const size_t i = (size_t)gy * W + gx;
        logits[img + i] = logit;
        if (b < 2 && mask.valid[b]) {  // the learned mask of this map, as lr_mask_kernel computes it
            const int ok = logit > 0.0f && gx - (int)mask.wta[b][i] >= 0;
            mask.valid[b][i] = (uint8_t)ok;
            mask.disp[b][i] = ok ? mask.dsub[b][i] : -1.0f;
        }
    }
}

// --- workspace layout -------------------------------------------------------------
struct LrLayout {
    size_t a1, a2, a3, z, g4, gz3, gz2, gz1, part, loss, frag, fl, total;
    int nb4, nbc, npart_max;
};

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

static LrLayout lr_layout(int B, int H, int W, bool train)
{
    LrLayout L{};
    const size_t npx = (size_t)B * H * W;
    const int nb4 = B * ((W + T1 - 1) / T1) * ((H + T1 - 1) / T1);
    const int nbc = B * ((W + CT_W - 1) / CT_W) * ((H + CT_H - 1) / CT_H);
    L.nb4 = nb4;
    L.nbc = nbc;
    size_t o = 0;
    L.frag = o; o += al(FP_FRAGS * 16);
    L.fl = o; o += al(FP_FLOATS * 4);
    if (!train) {  // fused inference keeps activations on chip
        L.total = o;
        return L;
    }
    L.a1 = o; o += al(npx * 32);
    L.a2 = o; o += al(npx * 32);
    L.a3 = o; o += al(npx * 32);
    L.z = o; o += al(npx * 4);
    if (train) {
        L.g4 = o; o += al(npx * 4);
        L.gz3 = o; o += al(npx * 32);
        L.gz2 = o; o += al(npx * 32);
        L.gz1 = o; o += al(npx * 32);
        const size_t p4 = (size_t)nb4 * 145, p16 = (size_t)nbc * (16 * 16 * 9 + 16);
        L.part = o; o += al((p4 > p16 ? p4 : p16) * 4);
        L.loss = o; o += al((size_t)nb4 * 4);
    }
    L.total = o;
    return L;
}

size_t lrnet_forward_ws_bytes(int B, int H, int W) { return lr_layout(B, H, W, false).total; }

}  // namespace sf

using namespace sf;

extern "C" int sf_lrnet_nparams(void) { return LR_NP; }

extern "C" size_t sf_lrnet_workspace_bytes(int B, int H, int W, int train)
{
    if (B <= 0 || H <= 0 || W <= 0) return 0;
    return lr_layout(B, H, W, train != 0).total;
}

static int lr_check(const float *params, const float *feat, int B, int H, int W, void *ws,
                    size_t ws_bytes, bool train)
{
    SF_REQUIRE(params && feat && ws, SF_EINVAL, "sf_lrnet: NULL pointer");
    SF_REQUIRE(B > 0 && H > 0 && W > 0, SF_EINVAL, "sf_lrnet: B, H, W must be positive");
    SF_REQUIRE(B <= 65535 && (long long)B * H * W <= (1LL << 30), SF_EINVAL, "sf_lrnet: batch too large");
    SF_REQUIRE(ws_bytes >= lr_layout(B, H, W, train).total, SF_ENOMEM, "sf_lrnet: workspace too small");
    return SF_OK;
}

static int lr_forward(const float *params, const float *feat, int B, int H, int W, uint8_t *ws,
                      const LrLayout &L, float *logits, const uint8_t *label, float *g4,
                      float *loss_part, hipStream_t st)
{
    uint16_t *a1 = reinterpret_cast<uint16_t *>(ws + L.a1);
    uint16_t *a2 = reinterpret_cast<uint16_t *>(ws + L.a2);
    uint16_t *a3 = reinterpret_cast<uint16_t *>(ws + L.a3);
    dim3 g1((W + T1 - 1) / T1, (H + T1 - 1) / T1, B);
    dim3 gc((W + CT_W - 1) / CT_W, (H + CT_H - 1) / CT_H, B);
    {
        ProfScope prof("lrnet_l1", st);
        hipLaunchKernelGGL(l1_fwd_kernel, g1, dim3(256), 0, st, params,
                           reinterpret_cast<const float4 *>(feat), H, W, a1);
    }
    {
        ProfScope prof("lrnet_conv16", st);
        hipLaunchKernelGGL(conv16_mfma_kernel<false>, gc, dim3(256), 0, st, params, OFF_W2, OFF_B2,
                           a1, (const uint16_t *)nullptr, H, W, a2);
        hipLaunchKernelGGL(conv16_mfma_kernel<false>, gc, dim3(256), 0, st, params, OFF_W3, OFF_B3,
                           a2, (const uint16_t *)nullptr, H, W, a3);
    }
    const float inv_n = 1.0f / (float)((double)B * H * W);
    {
        ProfScope prof("lrnet_l4", st);
        hipLaunchKernelGGL(l4_fwd_kernel, g1, dim3(256), 0, st, params, a3, H, W, logits, label,
                           inv_n, g4, loss_part);
    }
    return launch_status("lrnet forward");
}

namespace sf {
void lrnet_pack_targets(uint8_t *ws, uint4 **frag, float **fl)
{
    const LrLayout L = lr_layout(1, 1, 1, false);  // the fragments do not depend on B, H, W
    *frag = reinterpret_cast<uint4 *>(ws + L.frag);
    *fl = reinterpret_cast<float *>(ws + L.fl);
}

int lrnet_forward(const float *params, const float *feat, int B, int H, int W, float *logits,
                  uint8_t *ws, hipStream_t st, const LrMaskOut *mask, bool prepacked)
{
    LrMaskOut mo{};
    if (mask) {
        if (B > 2) return fail(SF_EINVAL, "lrnet_forward: a mask needs at most 2 maps");
        mo = *mask;
    }
    const LrLayout L = lr_layout(B, H, W, false);
    uint4 *frag = reinterpret_cast<uint4 *>(ws + L.frag);
    float *fl = reinterpret_cast<float *>(ws + L.fl);
    if (!prepacked) {
        ProfScope prof("lrnet_pack", st);
        hipLaunchKernelGGL(pack_fused_kernel, dim3(FP_NSLOT), dim3(64), 0, st, params, frag, fl);
    }
    ProfScope prof("lrnet_fused", st);  // the fused inference launch alone
    dim3 g((W + FT_W - 1) / FT_W, (H + FT_H - 1) / FT_H, B);
    hipLaunchKernelGGL(lrnet_fused_kernel, g, dim3(64 * FT_NW), 0, st, frag, fl,
                       reinterpret_cast<const float4 *>(feat), H, W, logits, mo);
    return launch_status("lrnet_fused_kernel");
}

int launch_lr_mask(const float *logits, const int16_t *wta, const float *dsub, int H, int W,
                   uint8_t *valid, float *disp, hipStream_t st)
{
    const int n = H * W;
    ProfScope prof("lrnet_mask", st);
    hipLaunchKernelGGL(lr_mask_kernel, dim3((n + 255) / 256), dim3(256), 0, st, logits, wta, dsub, H,
                       W, valid, disp);
    return launch_status("lr_mask_kernel");
}
}  // namespace sf

extern "C" int sf_lrnet_forward(const float *params, const float *feat, int B, int H, int W,
                                float *logits, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = lr_check(params, feat, B, H, W, workspace, ws_bytes, false);
    if (rc) return rc;
    SF_REQUIRE(logits, SF_EINVAL, "sf_lrnet_forward: NULL logits");
    return lrnet_forward(params, feat, B, H, W, logits, static_cast<uint8_t *>(workspace),
                         as_stream(stream));
}

// --- forward without allocation ----------------------------------------------
// The fused inference needs only the packed weight fragments and biases as
// scratch (lr_layout(.., false): 13,568 bytes, independent of B, H, W).  For
// callers that cannot allocate, they live in a file-scope device array: each
// GPU holds its own copy, whose device address is looked up once per device
// (with that device current) and kept; host code never passes the array's
// name itself to a kernel.
constexpr size_t LR_SCRATCH_BYTES = 16384;
static __device__ __align__(256) uint8_t scratch[LR_SCRATCH_BYTES];

constexpr int LR_SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[LR_SCRATCH_MAX_DEVICES] = {};

static int lr_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("sf_lrnet_forward_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return SF_EHIP;
    }
    SF_REQUIRE(dev >= 0 && dev < LR_SCRATCH_MAX_DEVICES, SF_EUNSUPPORTED,
               "sf_lrnet_forward_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("sf_lrnet_forward_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return SF_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SF_OK;
}

extern "C" int sf_lrnet_forward_noalloc(const float *params, const float *feat, int B, int H, int W,
                                        float *logits, void *stream)
{
    clear_error();
    SF_REQUIRE(params && feat && logits, SF_EINVAL, "sf_lrnet_forward_noalloc: NULL pointer");
    SF_REQUIRE(B > 0 && H > 0 && W > 0, SF_EINVAL, "sf_lrnet_forward_noalloc: B, H, W must be positive");
    SF_REQUIRE(B <= 65535 && (long long)B * H * W <= (1LL << 30), SF_EINVAL,
               "sf_lrnet_forward_noalloc: batch too large");
    SF_REQUIRE(lr_layout(B, H, W, false).total <= LR_SCRATCH_BYTES, SF_ENOMEM,
               "sf_lrnet_forward_noalloc: scratch smaller than the weight fragments");
    void *scr = nullptr;
    const int rc = lr_scratch(&scr);
    if (rc) return rc;
    return lrnet_forward(params, feat, B, H, W, logits, static_cast<uint8_t *>(scr), as_stream(stream));
}

extern "C" int sf_lrnet_mask(const float *logits, const int16_t *wta, const float *dsub, int H,
                             int W, uint8_t *valid, float *disp, void *stream)
{
    clear_error();
    SF_REQUIRE(logits && wta && dsub && valid && disp, SF_EINVAL, "sf_lrnet_mask: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0 && (long long)H * W <= (1LL << 30), SF_EINVAL, "sf_lrnet_mask: bad size");
    return launch_lr_mask(logits, wta, dsub, H, W, valid, disp, as_stream(stream));
}

static int lr_backward(const float *params, const float *feat, const float *g4, int B, int H, int W,
                       uint8_t *ws, const LrLayout &L, float *grad, hipStream_t st);

extern "C" int sf_lrnet_grad(const float *params, const float *feat, const uint8_t *label, int B,
                             int H, int W, float *grad, float *loss, void *workspace,
                             size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = lr_check(params, feat, B, H, W, workspace, ws_bytes, true);
    if (rc) return rc;
    SF_REQUIRE(label && grad && loss, SF_EINVAL, "sf_lrnet_grad: NULL pointer");
    hipStream_t st = as_stream(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    const LrLayout L = lr_layout(B, H, W, true);
    float *z = reinterpret_cast<float *>(ws + L.z);
    float *g4 = reinterpret_cast<float *>(ws + L.g4);
    float *lossp = reinterpret_cast<float *>(ws + L.loss);
    rc = lr_forward(params, feat, B, H, W, ws, L, z, label, g4, lossp, st);
    if (rc) return rc;
    rc = lr_backward(params, feat, g4, B, H, W, ws, L, grad, st);
    if (rc) return rc;
    ProfScope prof("lrnet_loss", st);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, lossp, L.nb4,
                       1.0f / (float)((double)B * H * W), loss);
    return launch_status("lrnet loss");
}

extern "C" int sf_lrnet_backward(const float *params, const float *feat, const float *dz4, int B,
                                 int H, int W, float *grad, void *workspace, size_t ws_bytes,
                                 void *stream)
{
    clear_error();
    int rc = lr_check(params, feat, B, H, W, workspace, ws_bytes, true);
    if (rc) return rc;
    SF_REQUIRE(dz4 && grad, SF_EINVAL, "sf_lrnet_backward: NULL pointer");
    hipStream_t st = as_stream(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    const LrLayout L = lr_layout(B, H, W, true);
    float *z = reinterpret_cast<float *>(ws + L.z);
    rc = lr_forward(params, feat, B, H, W, ws, L, z, nullptr, nullptr, nullptr, st);
    if (rc) return rc;
    return lr_backward(params, feat, dz4, B, H, W, ws, L, grad, st);
}

// Backward of the four layers from g4 = dL/dz4 [B][H][W], with the forward's
// BF16 activations a1..a3 in the workspace.
static int lr_backward(const float *params, const float *feat, const float *g4, int B, int H, int W,
                       uint8_t *ws, const LrLayout &L, float *grad, hipStream_t st)
{
    uint16_t *a1 = reinterpret_cast<uint16_t *>(ws + L.a1);
    uint16_t *a2 = reinterpret_cast<uint16_t *>(ws + L.a2);
    uint16_t *a3 = reinterpret_cast<uint16_t *>(ws + L.a3);
    uint16_t *gz3 = reinterpret_cast<uint16_t *>(ws + L.gz3);
    uint16_t *gz2 = reinterpret_cast<uint16_t *>(ws + L.gz2);
    uint16_t *gz1 = reinterpret_cast<uint16_t *>(ws + L.gz1);
    float *part = reinterpret_cast<float *>(ws + L.part);
    dim3 g1((W + T1 - 1) / T1, (H + T1 - 1) / T1, B);
    dim3 gc((W + CT_W - 1) / CT_W, (H + CT_H - 1) / CT_H, B);
    ProfScope prof("lrnet_bwd", st);
    // Layer 4.
    hipLaunchKernelGGL(l4_bwd_kernel, g1, dim3(256), 0, st, params, g4, a3, H, W, gz3, part);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(256), 0, st, part, L.nb4, 145, 144,
                       OFF_W4, OFF_B4, grad);
    // Layer 3: weight gradient, then the gradient w.r.t. the layer-2 pre-activation.
    hipLaunchKernelGGL(wgrad_mfma_kernel<16>, gc, dim3(256), 0, st, gz3, a2, (const float4 *)nullptr,
                       H, W, part);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(10), dim3(256), 0, st, part, L.nbc, 2320, 2304,
                       OFF_W3, OFF_B3, grad);
    hipLaunchKernelGGL(conv16_mfma_kernel<true>, gc, dim3(256), 0, st, params, OFF_W3, 0, gz3, a2, H,
                       W, gz2);
    // Layer 2.
    hipLaunchKernelGGL(wgrad_mfma_kernel<16>, gc, dim3(256), 0, st, gz2, a1, (const float4 *)nullptr,
                       H, W, part);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(10), dim3(256), 0, st, part, L.nbc, 2320, 2304,
                       OFF_W2, OFF_B2, grad);
    hipLaunchKernelGGL(conv16_mfma_kernel<true>, gc, dim3(256), 0, st, params, OFF_W2, 0, gz2, a1, H,
                       W, gz1);
    // Layer 1 (the features are the layer input).
    hipLaunchKernelGGL(wgrad_mfma_kernel<4>, gc, dim3(256), 0, st, gz1, (const uint16_t *)nullptr,
                       reinterpret_cast<const float4 *>(feat), H, W, part);
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(3), dim3(256), 0, st, part, L.nbc, 592, 576,
                       OFF_W1, OFF_B1, grad);
    return launch_status("lrnet backward");
}

extern "C" int sf_lrnet_adam(float *params, float *m, float *v, const float *grad, int n, float lr,
                             float b1, float b2, float eps, float b1t, float b2t, void *stream)
{
    clear_error();
    SF_REQUIRE(params && m && v && grad, SF_EINVAL, "sf_lrnet_adam: NULL pointer");
    SF_REQUIRE(n > 0, SF_EINVAL, "sf_lrnet_adam: n <= 0");
    SF_REQUIRE(b1t < 1.0f && b2t < 1.0f, SF_EINVAL, "sf_lrnet_adam: b1t, b2t must be < 1");
    ProfScope prof("lrnet_adam", as_stream(stream));
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), params,
                       m, v, grad, n, lr, b1, b2, eps, b1t, b2t);
    return launch_status("adam_kernel");
}
