// Machine-balance probes: the streaming rates of HBM (read, write, copy) and
// the packed 16-bit VALU rate, the two ceilings the stereo kernels are judged
// against.  Not part of the method.
#include "sf_internal.hpp"

namespace sf {

constexpr int PR_NT = 256;
constexpr int PR_U = 4;  // 16-byte vectors per thread per iteration

// mode 0: dst = src, 1: read src, 2: fill dst.  Each thread issues PR_U
// independent 16-byte accesses per iteration (grid-stride over groups).
template <int MODE>
__global__ __launch_bounds__(PR_NT) void stream_kernel(const u32x4 *__restrict__ src,
                                                       u32x4 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * PR_NT;
    const size_t chunk = (size_t)PR_NT * PR_U;           // vectors per block-iteration
    const size_t ng = (n + chunk - 1) / chunk * PR_NT;   // thread-iterations covering n
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (size_t g = (size_t)blockIdx.x * PR_NT + threadIdx.x; g < ng; g += stride) {
        const size_t base = (g / PR_NT) * chunk + g % PR_NT;  // lanes contiguous per vector
        u32x4 v[PR_U];
#pragma unroll
        for (int u = 0; u < PR_U; ++u) {
            const size_t i = base + (size_t)u * PR_NT;
            if (MODE == 2)
                v[u] = u32x4{(uint32_t)i, 1u, 2u, 3u};
            else if (i < n)
                v[u] = __builtin_nontemporal_load(src + i);
            else
                v[u] = u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < PR_U; ++u) {
            const size_t i = base + (size_t)u * PR_NT;
            if (MODE == 1)
                acc ^= v[u];
            else if (i < n)
                __builtin_nontemporal_store(v[u], dst + i);
        }
    }
    if (MODE == 1) asm volatile("" ::"v"(acc.x), "v"(acc.y), "v"(acc.z), "v"(acc.w));
}

// 16 packed 16-bit instructions (8 adds, 8 mins) per iteration over eight
// interleaved chains.
__global__ __launch_bounds__(PR_NT) void pk_u16_kernel(uint32_t *__restrict__ out, int iters, uint32_t seed)
{
    const uint32_t gid = blockIdx.x * PR_NT + threadIdx.x;
    u16x2 a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = as_u16x2(seed * (gid + 7u * k + 1u));
    const u16x2 b = as_u16x2(seed ^ gid);
    for (int it = 0; it < iters; ++it) {
        u16x2 t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = a[k] + b;
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_elementwise_min(t[k], t[(k + 1) & 7]);
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r ^= as_u32(a[k]);
    out[gid] = r;
}

}  // namespace sf

using namespace sf;

extern "C" int sf_probe_stream(const void *src, void *dst, size_t bytes, int mode, void *stream)
{
    clear_error();
    SF_REQUIRE(mode >= 0 && mode <= 2, SF_EINVAL, "sf_probe_stream: mode must be 0, 1 or 2");
    SF_REQUIRE(mode == 2 || src, SF_EINVAL, "sf_probe_stream: NULL src");
    SF_REQUIRE(mode == 1 || dst, SF_EINVAL, "sf_probe_stream: NULL dst");
    SF_REQUIRE(bytes % 16 == 0, SF_EINVAL, "sf_probe_stream: bytes must be a multiple of 16");
    SF_REQUIRE(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, SF_EINVAL,
               "sf_probe_stream: pointers must be 16-byte aligned");
    const size_t n = bytes / 16;
    if (n == 0) return SF_OK;
    const size_t chunks = (n + (size_t)PR_NT * PR_U - 1) / ((size_t)PR_NT * PR_U);
    const unsigned blocks = (unsigned)std::min<size_t>(chunks, 16384);
    hipStream_t st = as_stream(stream);
    const u32x4 *s = static_cast<const u32x4 *>(src);
    u32x4 *d = static_cast<u32x4 *>(dst);
    if (mode == 0)
        hipLaunchKernelGGL(stream_kernel<0>, dim3(blocks), dim3(PR_NT), 0, st, s, d, n);
    else if (mode == 1)
        hipLaunchKernelGGL(stream_kernel<1>, dim3(blocks), dim3(PR_NT), 0, st, s, d, n);
    else
        hipLaunchKernelGGL(stream_kernel<2>, dim3(blocks), dim3(PR_NT), 0, st, s, d, n);
    return launch_status("stream_kernel");
}

extern "C" int sf_probe_pk_u16(uint32_t *out, int blocks, int iters, void *stream)
{
    clear_error();
    SF_REQUIRE(out, SF_EINVAL, "sf_probe_pk_u16: NULL out");
    SF_REQUIRE(blocks > 0 && iters >= 0, SF_EINVAL, "sf_probe_pk_u16: blocks must be > 0, iters >= 0");
    hipLaunchKernelGGL(pk_u16_kernel, dim3(blocks), dim3(PR_NT), 0, as_stream(stream), out, iters,
                       0x9E3779B9u);
    return launch_status("pk_u16_kernel");
}
