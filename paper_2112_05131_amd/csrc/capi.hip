// capi.hip -- error state, validation and host-only entry points of the
// C ABI (plenoxel.h).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "plx_internal.hpp"

namespace plx {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PLX_EDEVICE, "%s: launch failed: %s", what, hipGetErrorString(e));
    return PLX_OK;
}

int validate_grid(const plx_grid *g, bool need_occ, const char *fn) {
    if (!g) return fail(PLX_EINVAL, "%s: grid is NULL", fn);
    for (int a = 0; a < 3; ++a)
        if (g->reso[a] < 2)
            return fail(PLX_EINVAL, "%s: reso[%d] = %d (need >= 2)", fn, a, g->reso[a]);
    if (n_cells(g->reso) > ((int64_t)1 << 34))
        return fail(PLX_EINVAL, "%s: grid of %lld cells is too large", fn,
                    (long long)n_cells(g->reso));
    if (g->n_vox < 0 || g->n_vox > (int64_t)0x7fffffff)
        return fail(PLX_EINVAL, "%s: n_vox = %lld out of range", fn, (long long)g->n_vox);
    if (g->n_vox > n_cells(g->reso))
        return fail(PLX_EINVAL, "%s: n_vox = %lld exceeds the number of cells", fn,
                    (long long)g->n_vox);
    if (g->sh_dtype != PLX_F32 && g->sh_dtype != PLX_BF16 && g->sh_dtype != PLX_F16)
        return fail(PLX_EINVAL, "%s: unknown sh_dtype %d", fn, g->sh_dtype);
    if (!g->index) return fail(PLX_EINVAL, "%s: grid index is NULL", fn);
    if (g->n_vox > 0 && !g->data) return fail(PLX_EINVAL, "%s: grid data is NULL", fn);
    if (need_occ && !g->occ) return fail(PLX_EINVAL, "%s: grid occupancy bitmap is NULL", fn);
    for (int a = 0; a < 3; ++a)
        if (!(g->scale[a] > 0.0f) || !isfinite(g->scale[a]) || !isfinite(g->offset[a]))
            return fail(PLX_EINVAL, "%s: bad scale/offset on axis %d", fn, a);
    if (!(g->step > 0.0f) || !isfinite(g->step))
        return fail(PLX_EINVAL, "%s: step must be positive and finite", fn);
    if ((reinterpret_cast<uintptr_t>(g->data) & 127u) != 0 && g->sh_dtype == PLX_F32)
        return fail(PLX_EINVAL, "%s: FP32 records must be 128-byte aligned", fn);
    if ((reinterpret_cast<uintptr_t>(g->data) & 63u) != 0)
        return fail(PLX_EINVAL, "%s: records must be 64-byte aligned", fn);
    return PLX_OK;
}

}  // namespace plx

using namespace plx;

extern "C" {

const char *plx_last_error(void) { return g_err; }

const char *plx_version(void) { return "plenoxel-hip 0.1 (gfx950)"; }

int64_t plx_record_bytes(int32_t sh_dtype) {
    switch (sh_dtype) {
    case PLX_F32: return kRecF32Bytes;
    case PLX_BF16:
    case PLX_F16: return kRec16Bytes;
    default: return 0;
    }
}

int64_t plx_occ_words(const int32_t reso[3]) {
    if (!reso) return 0;
    return occ_words(reso);
}

int64_t plx_occ_brick_offset(const int32_t reso[3]) {
    if (!reso || reso[0] < 2 || reso[1] < 2 || reso[2] < 2) return 0;
    return occ_brick_offset(reso);
}

int64_t plx_occ_bytes(const int32_t reso[3]) {
    if (!reso || reso[0] < 2 || reso[1] < 2 || reso[2] < 2) return 0;
    return (occ_brick_offset(reso) + n_bricks(reso) + 255) / 256 * 256;
}

int plx_grid_geometry(const int32_t reso[3], const double lo[3], const double hi[3],
                      double step_voxels, float scale_out[3], float offset_out[3],
                      float *step_out) {
    if (!reso || !lo || !hi || !scale_out || !offset_out || !step_out)
        return fail(PLX_EINVAL, "plx_grid_geometry: NULL argument");
    if (!(step_voxels > 0.0)) return fail(PLX_EINVAL, "plx_grid_geometry: step_voxels <= 0");
    double max_scale = 0.0;
    float sc[3], of[3];
    for (int a = 0; a < 3; ++a) {
        if (reso[a] < 2) return fail(PLX_EINVAL, "plx_grid_geometry: reso[%d] < 2", a);
        if (!(hi[a] > lo[a])) return fail(PLX_EINVAL, "plx_grid_geometry: empty box on axis %d", a);
        double s = (double)reso[a] / (hi[a] - lo[a]);
        sc[a] = (float)s;
        of[a] = (float)(-lo[a] * s - 0.5);
        if (s > max_scale) max_scale = s;
    }
    for (int a = 0; a < 3; ++a) {
        scale_out[a] = sc[a];
        offset_out[a] = of[a];
    }
    *step_out = (float)(step_voxels / max_scale);
    return PLX_OK;
}

double plx_lr_schedule(double step, double lr0, double lr1, double max_steps,
                       double delay_steps, double delay_mult) {
    double frac = max_steps > 0.0 ? step / max_steps : 1.0;
    frac = frac < 0.0 ? 0.0 : (frac > 1.0 ? 1.0 : frac);
    double lr = exp(log(lr0) * (1.0 - frac) + log(lr1) * frac);
    if (delay_steps > 0.0) {
        double u = step / delay_steps;
        u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
        lr *= delay_mult + (1.0 - delay_mult) * sin(0.5 * M_PI * u);
    }
    return lr;
}

}  // extern "C"
