// rays.hip -- the NDC warp of forward-facing rays (Sec. 3.6: forward-facing
// scenes use the normalized device coordinates derived in the NeRF paper)
// for gfx950.
//
// One ray per thread, FP64 in a fixed operation order without contraction,
// rounded to FP32 once: the warped rays are then the same bits wherever the
// warp is computed, so the samples, cells and touched sets of a render in NDC
// space are reproducible.
#include <cmath>

#include "plx_internal.hpp"

namespace plx {
namespace {

__global__ __launch_bounds__(256) void ndc_kernel(const float *rays_o, const float *rays_d, int64_t n,
                                                  double ax, double ay, double near, float *o_out,
                                                  float *d_out) {
#pragma clang fp contract(off)
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double o[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o[a] = (double)rays_o[3 * r + a];
        d[a] = (double)rays_d[3 * r + a];
    }
    if (d[2] == 0.0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) o_out[3 * r + a] = d_out[3 * r + a] = 0.0f;
        return;
    }
    // move the origin to the near plane z = -near
    const double t = -(near + o[2]) / d[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = o[a] + t * d[a];
    double op[3], dp[3];
    op[0] = ax * (o[0] / o[2]);
    op[1] = ay * (o[1] / o[2]);
    op[2] = 1.0 + 2.0 * near / o[2];
    dp[0] = ax * (d[0] / d[2] - o[0] / o[2]);
    dp[1] = ay * (d[1] / d[2] - o[1] / o[2]);
    dp[2] = -2.0 * near / o[2];
    const double nrm = sqrt(dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o_out[3 * r + a] = (float)op[a];
        d_out[3 * r + a] = (float)(dp[a] / nrm);
    }
}

}  // namespace
}  // namespace plx

using namespace plx;

extern "C" {

int plx_rays_to_ndc(const float *rays_o, const float *rays_d, int64_t n_rays, int32_t width,
                    int32_t height, double focal, double near, float *o_out, float *d_out,
                    plx_stream stream) {
    const char *fn = "plx_rays_to_ndc";
    if (n_rays < 0 || n_rays > ((int64_t)1 << 34)) return fail(PLX_EINVAL, "%s: bad n_rays", fn);
    if (width < 1 || height < 1) return fail(PLX_EINVAL, "%s: width and height must be >= 1", fn);
    if (!(focal > 0.0) || !std::isfinite(focal) || !(near > 0.0) || !std::isfinite(near))
        return fail(PLX_EINVAL, "%s: focal and near must be finite and > 0", fn);
    if (n_rays == 0) return PLX_OK;
    if (!rays_o || !rays_d || !o_out || !d_out) return fail(PLX_EINVAL, "%s: NULL array", fn);
    const double ax = -(2.0 * focal / (double)width);
    const double ay = -(2.0 * focal / (double)height);
    const int64_t nb = (n_rays + 255) / 256;
    ndc_kernel<<<(unsigned)nb, 256, 0, as_stream(stream)>>>(rays_o, rays_d, n_rays, ax, ay, near,
                                                            o_out, d_out);
    return check_launch(fn);
}

}  // extern "C"
