// Agreement of two validity masks: the judge of the learned stand-in against
// the left-right check it imitates (paper Sec. 3.1: the check compares two
// computed disparity maps; the learned mask predicts its outcome).  One block
// of 1024 threads counts the pixels whose two masks agree (both zero or both
// nonzero) and writes the count: no atomics, no clearing, the same count on
// every run.  16-byte loads when both masks are 16-byte aligned.
#include "sf_internal.hpp"

namespace sf {

constexpr int JUDGE_NT = 1024;

__device__ __forceinline__ uint32_t agree_bytes(uint32_t a, uint32_t b)
{
    // Number of the four byte positions where both bytes are zero or both nonzero.
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t ab = (a >> (8 * k)) & 0xFFu, bb = (b >> (8 * k)) & 0xFFu;
        n += ((ab != 0u) == (bb != 0u)) ? 1u : 0u;
    }
    return n;
}

__global__ __launch_bounds__(JUDGE_NT) void mask_agreement_kernel(const uint8_t *__restrict__ a,
                                                                  const uint8_t *__restrict__ b,
                                                                  int n, int vec, uint32_t *__restrict__ count)
{
    __shared__ uint32_t s_part[JUDGE_NT / 64];
    uint32_t c = 0;
    int tail = 0;
    if (vec) {
        const int nv = n / 16;
        const uint4 *a4 = reinterpret_cast<const uint4 *>(a);
        const uint4 *b4 = reinterpret_cast<const uint4 *>(b);
        for (int i = threadIdx.x; i < nv; i += JUDGE_NT) {
            const uint4 va = a4[i], vb = b4[i];
            c += agree_bytes(va.x, vb.x) + agree_bytes(va.y, vb.y) + agree_bytes(va.z, vb.z) +
                 agree_bytes(va.w, vb.w);
        }
        tail = nv * 16;
    }
    for (int i = tail + threadIdx.x; i < n; i += JUDGE_NT) c += ((a[i] != 0) == (b[i] != 0)) ? 1u : 0u;
    // Wave sum, then the block's 16 wave sums in order.
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < JUDGE_NT / 64; ++w) t += s_part[w];
        *count = t;
    }
}

}  // namespace sf

using namespace sf;

extern "C" int sf_mask_agreement(const uint8_t *a, const uint8_t *b, int n, uint32_t *count, void *stream)
{
    clear_error();
    SF_REQUIRE(a && b && count, SF_EINVAL, "sf_mask_agreement: NULL pointer");
    SF_REQUIRE(n > 0, SF_EINVAL, "sf_mask_agreement: n must be positive");
    const int vec = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
    ProfScope prof("mask_agreement", as_stream(stream));
    hipLaunchKernelGGL(mask_agreement_kernel, dim3(1), dim3(JUDGE_NT), 0, as_stream(stream), a, b, n, vec,
                       count);
    return launch_status("mask_agreement_kernel");
}
