// Combination of the two disparity maps and the flow into the scene-flow map
// (paper Sec. 3.3: the case definition of S, the bilinear interpolation
// equation for D1 at x + F(x), and the 3-D reading of (u, v, d0, d1) through
// the camera).  One thread per pixel; flow and outputs are read / written as
// float2 / float4 / 3 x float, coalesced along rows.  Built without FMA
// contraction so every product and sum is the FP32 operation stated.
#include "sf_check.hpp"
#include "sf_internal.hpp"
#include "stages.hpp"

SF_CHECK_TU(combine)

namespace sf {

__global__ __launch_bounds__(256) void combine_kernel(
    const float *__restrict__ disp0, const uint8_t *__restrict__ valid0,
    const float *__restrict__ disp1, const uint8_t *__restrict__ valid1,
    const float2 *__restrict__ flow, int H, int W, int has_cam, sf_camera cam,
    float4 *__restrict__ sf4, uint8_t *__restrict__ valid, float *__restrict__ xyz0,
    float *__restrict__ motion)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= W) return;
    const size_t i = (size_t)y * W + x;
    const float2 uv = flow[i];
    const float xp = (float)x + uv.x;
    const float yp = (float)y + uv.y;
    bool defined = false;
    float d0 = 0.0f, d1 = 0.0f;
    if (valid0[i] && xp >= 0.0f && xp <= (float)(W - 1) && yp >= 0.0f && yp <= (float)(H - 1)) {
        const int x0 = (int)floorf(xp), y0 = (int)floorf(yp);
        const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
        const size_t i00 = (size_t)y0 * W + x0, i10 = (size_t)y0 * W + x1;
        const size_t i01 = (size_t)y1 * W + x0, i11 = (size_t)y1 * W + x1;
        SF_BOUNDS(x0 >= 0 && y0 >= 0 && x1 < W && y1 < H && x0 <= x1 && y0 <= y1, CHK_COMBINE_TAP);
        if (valid1[i00] && valid1[i10] && valid1[i01] && valid1[i11]) {
            const float fx = xp - (float)x0;
            const float fy = yp - (float)y0;
            const float t00 = (disp1[i00] * (1.0f - fx)) * (1.0f - fy);
            const float t10 = (disp1[i10] * fx) * (1.0f - fy);
            const float t01 = (disp1[i01] * (1.0f - fx)) * fy;
            const float t11 = (disp1[i11] * fx) * fy;
            d1 = ((t00 + t10) + t01) + t11;
            d0 = disp0[i];
            defined = true;
        }
    }
    const float nanv = __builtin_nanf("");
    uint8_t vb = 0;
    if (defined) {
        vb = 1;
        sf4[i] = make_float4(uv.x, uv.y, d0, d1);
    } else {
        sf4[i] = make_float4(nanv, nanv, nanv, nanv);
    }
    if (has_cam) {
        float o[6];
        if (defined && d0 > 0.0f && d1 > 0.0f) {
            vb |= 2;
            const float fB = cam.f * cam.B;
            const float Z0 = fB / d0;
            const float X0 = (((float)x - cam.cx) * Z0) / cam.f;
            const float Y0 = (((float)y - cam.cy) * Z0) / cam.f;
            const float Z1 = fB / d1;
            const float X1 = ((xp - cam.cx) * Z1) / cam.f;
            const float Y1 = ((yp - cam.cy) * Z1) / cam.f;
            o[0] = X0; o[1] = Y0; o[2] = Z0;
            o[3] = X1 - X0; o[4] = Y1 - Y0; o[5] = Z1 - Z0;
        } else {
            for (int k = 0; k < 6; ++k) o[k] = nanv;
        }
        xyz0[3 * i + 0] = o[0];
        xyz0[3 * i + 1] = o[1];
        xyz0[3 * i + 2] = o[2];
        motion[3 * i + 0] = o[3];
        motion[3 * i + 1] = o[4];
        motion[3 * i + 2] = o[5];
    }
    valid[i] = vb;
}

// Temporal validation over three time steps: S_a (t_k -> t_k+1) is kept at x
// iff the chained pixel q = floor(x + (u, v) + 0.5) at t_k+1 lies in the image,
// S_b (t_k+1 -> t_k+2) is defined there, and the flows and disparity changes
// agree within tau_f and tau_d (FP32, in this order).  One thread per pixel.
__global__ __launch_bounds__(256) void temporal_check_kernel(const float4 *__restrict__ a,
                                                             const uint8_t *__restrict__ va,
                                                             const float4 *__restrict__ b,
                                                             const uint8_t *__restrict__ vb, int H,
                                                             int W, float tau_f, float tau_d,
                                                             uint8_t *__restrict__ out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= H * W) return;
    const int y = i / W, x = i - y * W;
    uint8_t ok = 0;
    if (va[i] & 1) {
        const float4 s = a[i];
        const float xq = floorf(__fadd_rn((float)x, s.x) + 0.5f);
        const float yq = floorf(__fadd_rn((float)y, s.y) + 0.5f);
        if (xq >= 0.0f && xq <= (float)(W - 1) && yq >= 0.0f && yq <= (float)(H - 1)) {
            const size_t j = (size_t)yq * W + (size_t)xq;
            SF_BOUNDS(j < (size_t)H * W, CHK_TEMPORAL);
            if (vb[j] & 1) {
                const float4 t = b[j];
                const float ca = s.w - s.z, cb = t.w - t.z;
                ok = fabsf(s.x - t.x) <= tau_f && fabsf(s.y - t.y) <= tau_f && fabsf(ca - cb) <= tau_d;
            }
        }
    }
    out[i] = ok;
}

int launch_combine(const float *disp0, const uint8_t *valid0, const float *disp1,
                   const uint8_t *valid1, const float *flow, int H, int W, const sf_camera *cam,
                   float *sf4, uint8_t *valid, float *xyz0, float *motion, hipStream_t st)
{
    sf_camera c = cam ? *cam : sf_camera{0.0f, 0.0f, 0.0f, 0.0f};
    dim3 grid((W + 255) / 256, H);
    ProfScope prof("combine", st);
    hipLaunchKernelGGL(combine_kernel, grid, dim3(256), 0, st, disp0, valid0, disp1, valid1,
                       reinterpret_cast<const float2 *>(flow), H, W, cam ? 1 : 0, c,
                       reinterpret_cast<float4 *>(sf4), valid, xyz0, motion);
    return launch_status("combine_kernel");
}

}  // namespace sf

using namespace sf;

extern "C" int sf_combine(const float *disp0, const uint8_t *valid0, const float *disp1,
                          const uint8_t *valid1, const float *flow, int H, int W,
                          const sf_camera *cam, float *sf4, uint8_t *valid, float *xyz0,
                          float *motion, void *stream)
{
    clear_error();
    SF_REQUIRE(disp0 && valid0 && disp1 && valid1 && flow && sf4 && valid, SF_EINVAL,
               "sf_combine: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_combine: H and W must be positive");
    SF_REQUIRE(H <= 65535, SF_EINVAL, "sf_combine: H > 65535");
    SF_REQUIRE(!cam || (xyz0 && motion), SF_EINVAL, "sf_combine: camera given without xyz0/motion");
    if (cam) SF_REQUIRE(cam->f != 0.0f, SF_EINVAL, "sf_combine: focal length is zero");
    return launch_combine(disp0, valid0, disp1, valid1, flow, H, W, cam, sf4, valid, xyz0, motion,
                          as_stream(stream));
}

extern "C" int sf_temporal_check(const float *sf4_a, const uint8_t *valid_a, const float *sf4_b,
                                 const uint8_t *valid_b, int H, int W, float tau_f, float tau_d,
                                 uint8_t *out, void *stream)
{
    clear_error();
    SF_REQUIRE(sf4_a && valid_a && sf4_b && valid_b && out, SF_EINVAL, "sf_temporal_check: NULL pointer");
    SF_REQUIRE(H > 0 && W > 0 && (long long)H * W <= (1LL << 30), SF_EINVAL,
               "sf_temporal_check: bad image size");
    SF_REQUIRE(tau_f >= 0.0f && tau_d >= 0.0f, SF_EINVAL, "sf_temporal_check: negative tolerance");
    SF_REQUIRE((reinterpret_cast<uintptr_t>(sf4_a) | reinterpret_cast<uintptr_t>(sf4_b)) % 16 == 0,
               SF_EINVAL, "sf_temporal_check: sf4 buffers must be 16-byte aligned");
    const int n = H * W;
    hipLaunchKernelGGL(temporal_check_kernel, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream),
                       reinterpret_cast<const float4 *>(sf4_a), valid_a,
                       reinterpret_cast<const float4 *>(sf4_b), valid_b, H, W, tau_f, tau_d, out);
    return launch_status("temporal_check_kernel");
}
