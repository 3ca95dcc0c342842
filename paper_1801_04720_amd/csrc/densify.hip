// Densification of the sparse scene-flow map.  The paper evaluates a dense
// version produced by the benchmark's own interpolation and names a better
// interpolation as future work (Sec. 4); the fill rule here is this library's:
//   * an undefined pixel takes (u, v, d0, d1) from the nearest defined pixel to
//     its left or right in the same row, the one with the smaller d0 (farther
//     surface) when both exist, ties to the left;
//   * a row without a defined pixel copies the nearest row that has one (ties
//     to the row above).
// Row pass: one block per row; each thread scans a contiguous segment for its
// first / last defined pixel, the block combines the segments, and the
// nearest-left / nearest-right index of every pixel lands in LDS.  Copy pass:
// one block per empty row.
#include "sf_check.hpp"
#include "sf_internal.hpp"

SF_CHECK_TU(densify)

namespace sf {

constexpr int DN_NT = 256;
constexpr int DN_MAXW = 8192;

__global__ __launch_bounds__(DN_NT) void densify_rows_kernel(const float4 *__restrict__ sf4,
                                                             const uint8_t *__restrict__ valid,
                                                             int W, float4 *__restrict__ out,
                                                             uint8_t *__restrict__ fill,
                                                             uint8_t *__restrict__ rowok)
{
    __shared__ int s_last[DN_NT], s_first[DN_NT];
    __shared__ int16_t s_nl[DN_MAXW], s_nr[DN_MAXW];
    const int y = blockIdx.x, t = threadIdx.x;
    const size_t row = (size_t)y * W;
    const int seg = (W + DN_NT - 1) / DN_NT;
    const int x0 = min(W, t * seg), x1 = min(W, x0 + seg);
    int last = -1, first = W;
    for (int x = x0; x < x1; ++x)
        if (valid[row + x] & 1) {
            if (first == W) first = x;
            last = x;
        }
    s_last[t] = last;
    s_first[t] = first;
    __syncthreads();
    // Nearest defined pixel before this segment and after it.
    int left = -1, right = W;
    for (int k = 0; k < t; ++k) left = max(left, s_last[k]);
    for (int k = DN_NT - 1; k > t; --k) right = min(right, s_first[k]);
    int cur = left;
    for (int x = x0; x < x1; ++x) {
        if (valid[row + x] & 1) cur = x;
        s_nl[x] = (int16_t)cur;  // nearest defined at or left of x
    }
    cur = right;
    for (int x = x1 - 1; x >= x0; --x) {
        if (valid[row + x] & 1) cur = x;
        s_nr[x] = (int16_t)cur;  // nearest defined at or right of x (W: none)
    }
    __syncthreads();
    const bool any = s_nl[W - 1] >= 0;
    const float nanv = __builtin_nanf("");
    for (int x = t; x < W; x += DN_NT) {
        float4 v = make_float4(nanv, nanv, nanv, nanv);
        uint8_t f = 0;
        if (valid[row + x] & 1) {
            v = sf4[row + x];
            f = 1;
        } else if (any) {
            const int xl = s_nl[x], xr = s_nr[x];
            int src;
            if (xl >= 0 && xr < W)
                src = (sf4[row + xr].z < sf4[row + xl].z) ? xr : xl;
            else
                src = xl >= 0 ? xl : xr;
            SF_BOUNDS(src >= 0 && src < W, CHK_DENSIFY);
            v = sf4[row + src];
            f = 2;
        }
        out[row + x] = v;
        fill[row + x] = f;
    }
    if (t == 0) rowok[y] = any ? 1 : 0;
}

__global__ __launch_bounds__(DN_NT) void densify_copy_rows_kernel(const uint8_t *__restrict__ rowok,
                                                                  int H, int W,
                                                                  float4 *__restrict__ out,
                                                                  uint8_t *__restrict__ fill)
{
    const int y = blockIdx.x;
    if (rowok[y]) return;
    int src = -1;
    for (int dy = 1; dy < H && src < 0; ++dy) {
        if (y - dy >= 0 && rowok[y - dy])
            src = y - dy;
        else if (y + dy < H && rowok[y + dy])
            src = y + dy;
    }
    if (src < 0) return;  // nothing defined anywhere: the row pass left NaN / 0
    SF_BOUNDS(src < H, CHK_DENSIFY);
    for (int x = threadIdx.x; x < W; x += DN_NT) {
        out[(size_t)y * W + x] = out[(size_t)src * W + x];
        fill[(size_t)y * W + x] = 3;
    }
}

}  // namespace sf

using namespace sf;

extern "C" size_t sf_densify_workspace_bytes(int H) { return H > 0 ? (size_t)H : 0; }

extern "C" int sf_densify(const float *sf4, const uint8_t *valid, int H, int W, float *out,
                          uint8_t *fill, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(sf4 && valid && out && fill, SF_EINVAL, "sf_densify: NULL pointer");
    SF_REQUIRE(sf4 != out, SF_EINVAL, "sf_densify: sf4 and out must not be the same buffer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_densify: H and W must be positive");
    SF_REQUIRE(W <= DN_MAXW, SF_EUNSUPPORTED, "sf_densify: W > 8192");
    SF_REQUIRE(workspace, SF_EINVAL, "sf_densify: NULL workspace");
    SF_REQUIRE(ws_bytes >= (size_t)H, SF_ENOMEM, "sf_densify: workspace too small");
    SF_REQUIRE((reinterpret_cast<uintptr_t>(sf4) | reinterpret_cast<uintptr_t>(out)) % 16 == 0,
               SF_EINVAL, "sf_densify: sf4 and out must be 16-byte aligned");
    hipStream_t st = as_stream(stream);
    uint8_t *rowok = static_cast<uint8_t *>(workspace);
    ProfScope prof("densify", st);
    hipLaunchKernelGGL(densify_rows_kernel, dim3(H), dim3(DN_NT), 0, st,
                       reinterpret_cast<const float4 *>(sf4), valid, W,
                       reinterpret_cast<float4 *>(out), fill, rowok);
    int rc = launch_status("densify_rows_kernel");
    if (rc) return rc;
    hipLaunchKernelGGL(densify_copy_rows_kernel, dim3(H), dim3(DN_NT), 0, st, rowok, H, W,
                       reinterpret_cast<float4 *>(out), fill);
    return launch_status("densify_copy_rows_kernel");
}
