// render.hip -- differentiable volume rendering over the sparse voxel grid
// (Sec. 3.1-3.3, Eq. (1); supplement B.1) for gfx950.
//
// Work mapping.  One ray per group of 8 lanes (8 rays per wave64, 32 per
// 256-thread block).  Lane L of a group owns record slots 4L..4L+3, so the 8
// lanes together read a voxel record with one 16-byte load each (one 128-byte
// line for FP32 records, half a line for 16-bit ones).  Lane 7 holds sigma
// (slot 28).  Ray-level scalars (geometry, transmittance, colour) are kept
// redundantly by the 8 lanes; SH colour is a 3-channel sum over the group
// (xor shuffles), sigma is a shuffle from lane 7.
//
// Exact empty-space skipping.  A sample whose lower-corner cell has no
// non-NULL corner reads only zeros: it changes neither colour nor
// transmittance and has no gradient.  Candidate samples are tested 32 at a
// time against the cell occupancy bitmap (4 per lane, one ballot each), and
// only the occupied ones are processed, in order.  The 8 corner ids and the
// lane's 8 corner values stay in registers while consecutive samples remain
// in the same cell.
//
// Backward.  The ray is replayed from its last sample to its first.  With
// tau_after the optical depth after sample k (starting from the forward
// total), T_{k+1} = exp(-tau_after), T_k = exp(-(tau_after - sigma delta))
// and the rest of the ray R_k = sum_{j>k} w_j c_j + T_n bg is a running sum;
// dC/dsigma_k = delta (T_{k+1} c_k - R_k), dC/dc_k = w_k.  Corner gradients
// are accumulated in registers while the ray stays in one cell and added to
// the FP32 gradient records with hardware float atomics when it leaves.
#include "plx_internal.hpp"

namespace plx {
namespace {

constexpr int kLPR = 8;                         // lanes per ray
constexpr int kThreads = 256;                   // 4 waves
constexpr int kRaysPerBlock = kThreads / kLPR;  // 32
constexpr int kChunk = 32;                      // candidate samples per round

enum { MODE_FWD = 0, MODE_BWD = 1, MODE_TRAIN = 2 };

struct RenderArgs {
    const float *rays_o;
    const float *rays_d;
    const float *target;    // TRAIN
    const float *grad_rgb;  // BWD
    const float *tau_in;    // BWD
    float *rgb_out;         // FWD (required), TRAIN (optional)
    float *tau_out;         // FWD (optional)
    float *grad;            // BWD, TRAIN
    uint32_t *touched;      // BWD, TRAIN
    double *loss_sum;       // TRAIN
    int64_t n_rays;
    float bg[3];
    float loss_scale;
    int n_blocks;
    int nb8;
};

// Per-lane corner cache of the current cell.
struct CornerCache {
    int64_t cell;  // storage id of the lower corner, -1 = none
    int myc;       // table id of corner L (this lane's corner)
    int ids[8];
    float4 val[8];
};

template <int DT>
__device__ inline void load_cell(const GridDev &g, int64_t lin, int L, CornerCache &cc) {
    const int64_t sy = g.nz, sx = (int64_t)g.ny * g.nz;
    const int64_t off = ((L >> 2) & 1) * sx + ((L >> 1) & 1) * sy + (L & 1);
    cc.cell = lin;
    cc.myc = g.index[lin + off];
#pragma unroll
    for (int c = 0; c < 8; ++c) cc.ids[c] = __shfl(cc.myc, c, kLPR);
#pragma unroll
    for (int c = 0; c < 8; ++c)
        cc.val[c] = cc.ids[c] >= 0 ? Rec<DT>::load4(g.data, cc.ids[c], L)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
}

__device__ inline void corner_weights(const float f[3], float w[8]) {
    const float ax[2] = {1.0f - f[0], f[0]};
    const float ay[2] = {1.0f - f[1], f[1]};
    const float az[2] = {1.0f - f[2], f[2]};
#pragma unroll
    for (int c = 0; c < 8; ++c) w[c] = ax[(c >> 2) & 1] * ay[(c >> 1) & 1] * az[c & 1];
}

// Interpolated slots of this lane, the (pre-ReLU) sigma of the group and the
// (pre-ReLU) colour of the group.
struct Interp {
    float sigma_pre;
    float col_pre[3];
};

__device__ inline Interp interpolate(const CornerCache &cc, const float w[8], const float yr[4],
                                     const float yg[4], const float yb[4]) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        v.x += w[c] * cc.val[c].x;
        v.y += w[c] * cc.val[c].y;
        v.z += w[c] * cc.val[c].z;
        v.w += w[c] * cc.val[c].w;
    }
    float pr = v.x * yr[0] + v.y * yr[1] + v.z * yr[2] + v.w * yr[3];
    float pg = v.x * yg[0] + v.y * yg[1] + v.z * yg[2] + v.w * yg[3];
    float pb = v.x * yb[0] + v.y * yb[1] + v.z * yb[2] + v.w * yb[3];
#pragma unroll
    for (int m = 1; m < kLPR; m <<= 1) {
        pr += __shfl_xor(pr, m, kLPR);
        pg += __shfl_xor(pg, m, kLPR);
        pb += __shfl_xor(pb, m, kLPR);
    }
    Interp r;
    r.sigma_pre = __shfl(v.x, 7, kLPR);
    r.col_pre[0] = pr;
    r.col_pre[1] = pg;
    r.col_pre[2] = pb;
    return r;
}

// Occupancy of the 32 candidate samples k0..k0+31 of the group's ray
// (bit i = sample k0+i lies in an occupied cell).  Group-uniform result.
__device__ inline uint32_t chunk_mask(const GridDev &g, const RayGeom &r, int n, int k0, int L) {
    uint32_t m = 0;
    const int shift = threadIdx.x & 56;
#pragma unroll
    for (int j = 0; j < kChunk / kLPR; ++j) {
        const int k = k0 + j * kLPR + L;
        bool ne = false;
        if (k < n) {
            Sample s = sample_at(g, r, k);
            ne = cell_occupied(g, cell_id(g, s.cell));
        }
        unsigned long long b = __ballot(ne);
        m |= ((uint32_t)(b >> shift) & 0xffu) << (kLPR * j);
    }
    return m;
}

// Adds the register accumulators of the cached cell into the gradient
// records and marks its non-NULL corners as touched.
__device__ inline void flush(float *grad, uint32_t *touched, const CornerCache &cc, float4 acc[8],
                             int L) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (cc.ids[c] >= 0) {
            float *p = grad + (int64_t)cc.ids[c] * PLX_REC_SLOTS + 4 * L;
            const float a4[4] = {acc[c].x, acc[c].y, acc[c].z, acc[c].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s = 4 * L + e;
                if ((s < PLX_NSH || s == PLX_SLOT_SIGMA) && a4[e] != 0.0f) unsafeAtomicAdd(p + e, a4[e]);
            }
        }
        acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (cc.myc >= 0) atomicOr(touched + (cc.myc >> 5), 1u << (cc.myc & 31));
}

template <int DT, int MODE>
__global__ __launch_bounds__(kThreads) void render_kernel(GridDev g, RenderArgs a) {
    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int L = threadIdx.x & (kLPR - 1);
    const int64_t ray = (int64_t)blk * kRaysPerBlock + (threadIdx.x / kLPR);
    const bool live = ray < a.n_rays;

    float o[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
    if (live) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            o[i] = a.rays_o[3 * ray + i];
            d[i] = a.rays_d[3 * ray + i];
        }
    }
    RayGeom r;
    const int n = live ? ray_setup(g, o, d, r) : 0;

    // SH basis of this lane's four slots, split by colour channel
    float yr[4], yg[4], yb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int s = 4 * L + e;
        const float y = s < PLX_NSH ? sh_basis_at(s % 9, d[0], d[1], d[2]) : 0.0f;
        const int ch = s / 9;
        yr[e] = ch == 0 ? y : 0.0f;
        yg[e] = ch == 1 ? y : 0.0f;
        yb[e] = (ch == 2 && s < PLX_NSH) ? y : 0.0f;
    }

    CornerCache cc;
    cc.cell = -1;
    cc.myc = -1;

    float C[3] = {0.f, 0.f, 0.f};
    float tau = 0.0f;
    double loss = 0.0;
    float gr[3] = {0.f, 0.f, 0.f};

    // ------------------------------------------------------------ forward
    if (MODE == MODE_FWD || MODE == MODE_TRAIN) {
        float T = 1.0f;
        for (int k0 = 0; k0 < n; k0 += kChunk) {
            uint32_t m = chunk_mask(g, r, n, k0, L);
            while (m) {
                const int bit = __ffs(m) - 1;
                m &= m - 1;
                const Sample s = sample_at(g, r, k0 + bit);
                const int64_t lin = cell_id(g, s.cell);
                if (lin != cc.cell) load_cell<DT>(g, lin, L, cc);
                float w[8];
                corner_weights(s.f, w);
                const Interp ip = interpolate(cc, w, yr, yg, yb);
                const float sigma = fmaxf(ip.sigma_pre, 0.0f);
                const float sd = sigma * s.delta;
                const float wk = T * (-expm1f(-sd));
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) C[ch] += wk * fmaxf(ip.col_pre[ch], 0.0f);
                T *= expf(-sd);
                tau += sd;
            }
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * a.bg[ch];
        if (live && L == 0) {
            if (MODE == MODE_FWD || a.rgb_out) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) a.rgb_out[3 * ray + ch] = C[ch];
            }
            if (MODE == MODE_FWD && a.tau_out) a.tau_out[ray] = tau;
        }
        if (MODE == MODE_TRAIN && live) {
            float l2 = 0.0f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float diff = C[ch] - a.target[3 * ray + ch];
                gr[ch] = 2.0f * a.loss_scale * diff;
                l2 += diff * diff;
            }
            if (L == 0) loss = (double)a.loss_scale * (double)l2;
        }
    }

    // ------------------------------------------------------------ backward
    if (MODE == MODE_BWD || MODE == MODE_TRAIN) {
        if (MODE == MODE_BWD && live) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gr[ch] = a.grad_rgb[3 * ray + ch];
            tau = a.tau_in[ray];
        }
        float4 acc[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
        bool dirty = false;
        float tau_after = tau;
        float T_after = expf(-tau_after);
        float gR = T_after * (gr[0] * a.bg[0] + gr[1] * a.bg[1] + gr[2] * a.bg[2]);
        const int last0 = n > 0 ? ((n - 1) / kChunk) * kChunk : -1;
        for (int k0 = last0; k0 >= 0; k0 -= kChunk) {
            uint32_t m = chunk_mask(g, r, n, k0, L);
            while (m) {
                const int bit = 31 - __clz(m);
                m &= ~(1u << bit);
                const Sample s = sample_at(g, r, k0 + bit);
                const int64_t lin = cell_id(g, s.cell);
                if (lin != cc.cell) {
                    if (dirty) flush(a.grad, a.touched, cc, acc, L);
                    load_cell<DT>(g, lin, L, cc);
                }
                dirty = true;
                float w[8];
                corner_weights(s.f, w);
                const Interp ip = interpolate(cc, w, yr, yg, yb);
                const float sigma = fmaxf(ip.sigma_pre, 0.0f);
                const float sd = sigma * s.delta;
                const float tau_before = fmaxf(tau_after - sd, 0.0f);
                const float T_before = expf(-tau_before);
                const float wk = T_before * (-expm1f(-sd));
                float col[3], gc = 0.0f;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    col[ch] = fmaxf(ip.col_pre[ch], 0.0f);
                    gc += gr[ch] * col[ch];
                }
                const float dsig = ip.sigma_pre > 0.0f ? s.delta * (T_after * gc - gR) : 0.0f;
                const float dR = ip.col_pre[0] > 0.0f ? wk * gr[0] : 0.0f;
                const float dG = ip.col_pre[1] > 0.0f ? wk * gr[1] : 0.0f;
                const float dB = ip.col_pre[2] > 0.0f ? wk * gr[2] : 0.0f;
                gR += wk * gc;
                tau_after = tau_before;
                T_after = T_before;
                // this lane's four slot gradients (slot 28 = sigma on lane 7)
                float dk[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) dk[e] = yr[e] * dR + yg[e] * dG + yb[e] * dB;
                if (L == 7) dk[0] = dsig;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    acc[c].x += w[c] * dk[0];
                    acc[c].y += w[c] * dk[1];
                    acc[c].z += w[c] * dk[2];
                    acc[c].w += w[c] * dk[3];
                }
            }
        }
        if (dirty) flush(a.grad, a.touched, cc, acc, L);
    }

    if (MODE == MODE_TRAIN) {
        // one double atomic per wave for the loss
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) loss += __shfl_xor(loss, m);
        if ((threadIdx.x & 63) == 0 && loss != 0.0) unsafeAtomicAdd(a.loss_sum, loss);
    }
}

// Work counters (one thread per ray; diagnostic, not a hot path).
__global__ void stats_kernel(GridDev g, const float *rays_o, const float *rays_d, int64_t n_rays,
                             uint32_t *cell_mark, uint32_t *vox_mark, unsigned long long *cnt) {
    const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long n_all = 0, n_occ = 0;
    if (ray < n_rays) {
        float o[3], d[3];
        for (int i = 0; i < 3; ++i) {
            o[i] = rays_o[3 * ray + i];
            d[i] = rays_d[3 * ray + i];
        }
        RayGeom r;
        const int n = ray_setup(g, o, d, r);
        n_all = n;
        int64_t last = -1;
        const int64_t sy = g.nz, sx = (int64_t)g.ny * g.nz;
        for (int k = 0; k < n; ++k) {
            const Sample s = sample_at(g, r, k);
            const int64_t lin = cell_id(g, s.cell);
            if (!cell_occupied(g, lin)) continue;
            ++n_occ;
            if (lin == last) continue;
            last = lin;
            for (int c = 0; c < 8; ++c) {
                const int64_t v = lin + ((c >> 2) & 1) * sx + ((c >> 1) & 1) * sy + (c & 1);
                atomicOr(cell_mark + (v >> 5), 1u << (v & 31));
                const int id = g.index[v];
                if (id >= 0) atomicOr(vox_mark + (id >> 5), 1u << (id & 31));
            }
        }
    }
    for (int m = 32; m >= 1; m >>= 1) {
        n_all += __shfl_xor(n_all, m);
        n_occ += __shfl_xor(n_occ, m);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&cnt[0], n_all);
        atomicAdd(&cnt[1], n_occ);
    }
}

int validate_rays(const float *o, const float *d, int64_t n, const char *fn) {
    if (n < 0) return fail(PLX_EINVAL, "%s: n_rays < 0", fn);
    if (n > ((int64_t)1 << 36)) return fail(PLX_EINVAL, "%s: n_rays too large", fn);
    if (n > 0 && (!o || !d)) return fail(PLX_EINVAL, "%s: rays are NULL", fn);
    return PLX_OK;
}

template <int MODE>
int launch_render(const plx_grid *grid, RenderArgs &a, hipStream_t s, const char *fn) {
    const int64_t nb = (a.n_rays + kRaysPerBlock - 1) / kRaysPerBlock;
    if (nb > 0x7ffffff0) return fail(PLX_EINVAL, "%s: too many rays", fn);
    a.n_blocks = (int)nb;
    a.nb8 = round_up8(nb);
    GridDev g = to_dev(grid);
    PLX_DISPATCH_DT(grid->sh_dtype, DT,
                    render_kernel<DT, MODE><<<a.nb8, kThreads, 0, s>>>(g, a));
    return check_launch(fn);
}

RenderArgs base_args(const plx_render_opts *opts, const float *o, const float *d, int64_t n) {
    RenderArgs a = {};
    a.rays_o = o;
    a.rays_d = d;
    a.n_rays = n;
    for (int i = 0; i < 3; ++i) a.bg[i] = opts->background[i];
    return a;
}

}  // namespace
}  // namespace plx

using namespace plx;

extern "C" {

int plx_render_fwd(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                   const float *rays_d, int64_t n_rays, float *rgb_out, float *tau_out,
                   plx_stream stream) {
    const char *fn = "plx_render_fwd";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!rgb_out) return fail(PLX_EINVAL, "%s: rgb_out is NULL", fn);
    RenderArgs a = base_args(opts, rays_o, rays_d, n_rays);
    a.rgb_out = rgb_out;
    a.tau_out = tau_out;
    return launch_render<MODE_FWD>(grid, a, as_stream(stream), fn);
}

int plx_render_bwd(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                   const float *rays_d, int64_t n_rays, const float *grad_rgb,
                   const float *tau_fwd, float *grad, uint32_t *touched, plx_stream stream) {
    const char *fn = "plx_render_bwd";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!grad_rgb || !tau_fwd || !grad || !touched)
        return fail(PLX_EINVAL, "%s: NULL grad_rgb/tau_fwd/grad/touched", fn);
    RenderArgs a = base_args(opts, rays_o, rays_d, n_rays);
    a.grad_rgb = grad_rgb;
    a.tau_in = tau_fwd;
    a.grad = grad;
    a.touched = touched;
    return launch_render<MODE_BWD>(grid, a, as_stream(stream), fn);
}

int plx_render_train(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                     const float *rays_d, const float *target, int64_t n_rays, float loss_scale,
                     float *rgb_out, float *grad, uint32_t *touched, double *loss_sum,
                     plx_stream stream) {
    const char *fn = "plx_render_train";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!target || !grad || !touched || !loss_sum)
        return fail(PLX_EINVAL, "%s: NULL target/grad/touched/loss_sum", fn);
    RenderArgs a = base_args(opts, rays_o, rays_d, n_rays);
    a.target = target;
    a.rgb_out = rgb_out;
    a.grad = grad;
    a.touched = touched;
    a.loss_sum = loss_sum;
    a.loss_scale = loss_scale;
    return launch_render<MODE_TRAIN>(grid, a, as_stream(stream), fn);
}

int plx_render_stats(const plx_grid *grid, const float *rays_o, const float *rays_d,
                     int64_t n_rays, uint32_t *cell_mark, uint32_t *vox_mark, int64_t counts[4],
                     plx_stream stream) {
    const char *fn = "plx_render_stats";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!cell_mark || !vox_mark || !counts) return fail(PLX_EINVAL, "%s: NULL argument", fn);
    hipStream_t s = as_stream(stream);
    const int64_t cw = plx_occ_words(grid->reso), vw = (grid->n_vox + 31) / 32;
    PLX_CHECK_HIP(hipMemsetAsync(cell_mark, 0, cw * 4, s), fn);
    if (vw) PLX_CHECK_HIP(hipMemsetAsync(vox_mark, 0, vw * 4, s), fn);
    TempBuf tmp;
    if ((rc = tmp.alloc(2 * sizeof(unsigned long long), s))) return rc;
    auto *cnt = static_cast<unsigned long long *>(tmp.ptr);
    PLX_CHECK_HIP(hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), s), fn);
    if (n_rays > 0) {
        stats_kernel<<<(unsigned)((n_rays + 255) / 256), 256, 0, s>>>(to_dev(grid), rays_o, rays_d,
                                                                      n_rays, cell_mark, vox_mark, cnt);
        if ((rc = check_launch(fn))) return rc;
    }
    unsigned long long h[2];
    PLX_CHECK_HIP(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s), fn);
    PLX_CHECK_HIP(hipStreamSynchronize(s), fn);
    counts[0] = (int64_t)h[0];
    counts[1] = (int64_t)h[1];
    int64_t cells = 0, vox = 0;
    if ((rc = plx_touched_count(cell_mark, n_cells(grid->reso), &cells, stream))) return rc;
    if ((rc = plx_touched_count(vox_mark, grid->n_vox, &vox, stream))) return rc;
    counts[2] = cells;
    counts[3] = vox;
    return PLX_OK;
}

}  // extern "C"
