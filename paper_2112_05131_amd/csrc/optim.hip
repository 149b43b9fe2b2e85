// optim.hip -- RMSProp with sparse (active-voxel) updates (Sec. 3.5 and
// Sec. 3.8: the gradient is very sparse, so only voxels that received a
// gradient term are updated) for gfx950.
//
// 8 lanes per voxel (32 voxels per 256-thread block), 4 FP32 slots per lane
// (16-byte accesses, one 128-byte line per voxel and array).  An inactive
// voxel costs one byte read of the touched map, so the cost of a step follows
// the active set, not the grid.
#include "plx_internal.hpp"

namespace plx {
namespace {

template <int DT>
__global__ __launch_bounds__(256) void rmsprop_kernel(void *data, float *master, float *vstate,
                                                      float *grad, uint8_t *touched,
                                                      int64_t n_vox, float lr_sigma, float lr_sh,
                                                      float beta, float eps) {
    const int L = threadIdx.x & 7;
    const int64_t m = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
    if (m >= n_vox) return;
    // the 8 lanes of a voxel (one wave) read its byte before lane 0 clears it
    if (!touched[m]) return;
    if (L == 0) touched[m] = 0;

    float *P = DT == PLX_F32 ? static_cast<float *>(data) : master;
    float4 *pp = reinterpret_cast<float4 *>(P + m * PLX_REC_SLOTS) + L;
    float4 *gp = reinterpret_cast<float4 *>(grad + m * PLX_REC_SLOTS) + L;
    float4 *vp = reinterpret_cast<float4 *>(vstate + m * PLX_REC_SLOTS) + L;
    float4 p4 = *pp, g4 = *gp, v4 = *vp;
    float p[4] = {p4.x, p4.y, p4.z, p4.w};
    const float gg[4] = {g4.x, g4.y, g4.z, g4.w};
    float v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int s = 4 * L + e;
        if (s < PLX_NSH || s == PLX_SLOT_SIGMA) {
            const float lr = s == PLX_SLOT_SIGMA ? lr_sigma : lr_sh;
            v[e] = beta * v[e] + (1.0f - beta) * gg[e] * gg[e];
            p[e] = p[e] - lr * gg[e] / (sqrtf(v[e]) + eps);
        }
    }
    *pp = make_float4(p[0], p[1], p[2], p[3]);
    *vp = make_float4(v[0], v[1], v[2], v[3]);
    *gp = make_float4(0.f, 0.f, 0.f, 0.f);
    if (DT != PLX_F32) {
        uint2 w;
        if (L == 7) {
            w.x = __float_as_uint(p[0]);
            w.y = 0u;
        } else {
            w.x = to16<DT>(p[0]) | (to16<DT>(p[1]) << 16);
            w.y = to16<DT>(p[2]) | (to16<DT>(p[3]) << 16);
            if (L == 6) w.y &= 0xffffu;
        }
        reinterpret_cast<uint2 *>(static_cast<char *>(data) + m * kRec16Bytes)[L] = w;
    }
}

}  // namespace
}  // namespace plx

using namespace plx;

extern "C" int plx_rmsprop_step(const plx_grid *grid, float *master, float *vstate, float *grad,
                                uint8_t *touched, float lr_sigma, float lr_sh, float beta,
                                float eps, plx_stream stream) {
    const char *fn = "plx_rmsprop_step";
    int rc = validate_grid(grid, false, fn);
    if (rc) return rc;
    if (grid->n_vox == 0) return PLX_OK;
    if (!vstate || !grad || !touched) return fail(PLX_EINVAL, "%s: NULL vstate/grad/touched", fn);
    if (grid->sh_dtype == PLX_F32 && master)
        return fail(PLX_EINVAL, "%s: master must be NULL for FP32 grids", fn);
    if (grid->sh_dtype != PLX_F32 && !master)
        return fail(PLX_EINVAL, "%s: 16-bit grids need the FP32 master records", fn);
    if (!(beta >= 0.0f && beta < 1.0f)) return fail(PLX_EINVAL, "%s: beta must be in [0, 1)", fn);
    const int64_t nw = (grid->n_vox + 31) / 32;
    if (nw > 0x7fffffff) return fail(PLX_EINVAL, "%s: grid too large", fn);
    hipStream_t s = as_stream(stream);
    PLX_DISPATCH_DT(grid->sh_dtype, DT,
                    rmsprop_kernel<DT><<<(unsigned)nw, 256, 0, s>>>(grid->data, master, vstate, grad,
                                                                    touched, grid->n_vox, lr_sigma,
                                                                    lr_sh, beta, eps));
    return check_launch(fn);
}
