// tv.hip -- total-variation regulariser over a contiguous segment of cells
// (Sec. 3.5, the loss below Eq. (2); supplement B.1: stochastic TV on
// random contiguous segments of the pointer grid, differences normalised by
// D/256, and the SH rule that empty cells and edges count as equal to the
// current cell) for gfx950.
//
// Density term: one thread per cell of the segment, reading the cell and
// its three forward neighbours (NULL or out of range = 0).  SH terms exist
// only for a non-NULL cell (a NULL or out-of-range neighbour gives a zero
// difference): the block collects its non-NULL cells in LDS and then handles
// each with 32 lanes, lane q = coefficient q, so the four records are read and
// the four gradient records updated with one line-wide access each.
// The MSI background's instance uses its three colour coefficients as the
// colour terms and wraps its last (azimuth) axis.
// Gradients go to the cell and its neighbours with float atomics
// (neighbouring cells share voxels); the loss is reduced per block and added
// once in FP64.
#include "plx_internal.hpp"

namespace plx {
namespace {

// BG: the MSI background grid's TV, whose colour terms are its three colour
// coefficients (record slots 24-26) and whose last (azimuth) axis wraps.
constexpr int kBgSlot = 24;

template <int DT, bool BG>
__global__ __launch_bounds__(256) void tv_kernel(GridDev g, int64_t start, int64_t count,
                                                 int64_t ncell, float lam_sig_v, float lam_sh_v,
                                                 float eps, float s0, float s1, float s2,
                                                 float *grad, uint8_t *touched, double *loss_sum) {
    __shared__ int4 cells[256];  // non-NULL cells of the block: id and forward neighbours
    __shared__ int n_cells_sh;
    __shared__ double part[4];
    if (threadIdx.x == 0) n_cells_sh = 0;
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float sa[3] = {s0, s1, s2};
    double local = 0.0;
    if (c < count) {
        int64_t v = start + c;
        v = v < ncell ? v : v % ncell;
        const int k = (int)(v % g.nz);
        const int64_t r = v / g.nz;
        const int j = (int)(r % g.ny);
        const int i = (int)(r / g.ny);
        const int64_t sy = g.nz, sx = (int64_t)g.ny * g.nz;
        const int id = g.index[v];
        const int nid[3] = {i + 1 < g.nx ? g.index[v + sx] : -1, j + 1 < g.ny ? g.index[v + sy] : -1,
                            k + 1 < g.nz ? g.index[v + 1] : (BG ? g.index[v - k] : -1)};

        // density channel: NULL or out-of-range reads 0
        {
            const float x0 = id >= 0 ? rec_sigma<DT>(g.data, id) : 0.0f;
            float dl[3], ss = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float xa = nid[a] >= 0 ? rec_sigma<DT>(g.data, nid[a]) : 0.0f;
                dl[a] = sa[a] * (xa - x0);
                ss += dl[a] * dl[a];
            }
            const float term = sqrtf(ss + eps);
            local += (double)lam_sig_v * (double)term;
            const float coef = lam_sig_v / term;
            if (id >= 0) {
                const float gsum = sa[0] * dl[0] + sa[1] * dl[1] + sa[2] * dl[2];
                const float gv = -coef * gsum;
                if (gv != 0.0f) unsafeAtomicAdd(grad + (int64_t)id * PLX_REC_SLOTS + PLX_SLOT_SIGMA, gv);
                touched[id] = 1;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (nid[a] < 0) continue;
                const float gv = coef * sa[a] * dl[a];
                if (gv != 0.0f)
                    unsafeAtomicAdd(grad + (int64_t)nid[a] * PLX_REC_SLOTS + PLX_SLOT_SIGMA, gv);
                touched[nid[a]] = 1;
            }
        }
        if (id >= 0) cells[atomicAdd(&n_cells_sh, 1)] = make_int4(id, nid[0], nid[1], nid[2]);
    }
    __syncthreads();

    // SH channels of the non-NULL cells: 8 groups of 32 lanes, lane q = slot q
    const int q = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int nc = n_cells_sh;
    for (int e = grp; e < nc; e += 8) {
        const int4 cl = cells[e];
        const int nb[3] = {cl.y, cl.z, cl.w};
        float term = 0.0f;
        if (BG ? (q >= kBgSlot && q < kBgSlot + 3) : q < PLX_NSH) {
            const float x0 = rec_slot<DT>(g.data, cl.x, q);
            float dl[3], ss = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dl[a] = nb[a] >= 0 ? sa[a] * (rec_slot<DT>(g.data, nb[a], q) - x0) : 0.0f;
                ss += dl[a] * dl[a];
            }
            term = sqrtf(ss + eps);
            const float coef = lam_sh_v / term;
            float gsum = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (nb[a] < 0) continue;
                const float gv = coef * sa[a] * dl[a];
                gsum += sa[a] * dl[a];
                if (gv != 0.0f) unsafeAtomicAdd(grad + (int64_t)nb[a] * PLX_REC_SLOTS + q, gv);
            }
            const float gv = -coef * gsum;
            if (gv != 0.0f) unsafeAtomicAdd(grad + (int64_t)cl.x * PLX_REC_SLOTS + q, gv);
        }
        local += (double)lam_sh_v * (double)term;
    }

    // block reduction of the loss, one FP64 atomic per block
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) local += __shfl_xor(local, m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0 && loss_sum) {
        const double t = part[0] + part[1] + part[2] + part[3];
        if (t != 0.0) unsafeAtomicAdd(loss_sum, t);
    }
}

}  // namespace
}  // namespace plx

using namespace plx;

namespace plx {
namespace {

int tv_launch(const plx_grid *grid, int64_t cell_start, int64_t cell_count, float lambda_sigma,
              float lambda_sh, float eps, float *grad, uint8_t *touched, double *loss_sum,
              plx_stream stream, bool bg, const char *fn) {
    int rc = validate_grid(grid, false, fn);
    if (rc) return rc;
    if (bg && grid->sh_dtype != PLX_F32) return fail(PLX_EINVAL, "%s: background records must be FP32", fn);
    if (cell_count < 0) return fail(PLX_EINVAL, "%s: cell_count < 0", fn);
    if (cell_count == 0) return PLX_OK;
    if (!grad || !touched) return fail(PLX_EINVAL, "%s: grad/touched is NULL", fn);
    // eps > 0 keeps the square root and its derivative finite where all three
    // differences vanish (constant regions, the uniform initial grid)
    if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(PLX_EINVAL, "%s: eps must be positive and finite", fn);
    const int64_t ncell = n_cells(grid->reso);
    const int64_t start = ((cell_start % ncell) + ncell) % ncell;
    const float inv = (float)(1.0 / (double)cell_count);
    hipStream_t s = as_stream(stream);
    const unsigned nb = (unsigned)((cell_count + 255) / 256);
    GridDev g = to_dev(grid);
    const float s0 = grid->reso[0] / 256.0f, s1 = grid->reso[1] / 256.0f, s2 = grid->reso[2] / 256.0f;
    if (bg) {
        tv_kernel<PLX_F32, true><<<nb, 256, 0, s>>>(g, start, cell_count, ncell, lambda_sigma * inv,
                                                    lambda_sh * inv, eps, s0, s1, s2, grad, touched,
                                                    loss_sum);
    } else {
        PLX_DISPATCH_DT(grid->sh_dtype, DT,
                        tv_kernel<DT, false><<<nb, 256, 0, s>>>(g, start, cell_count, ncell,
                                                                lambda_sigma * inv, lambda_sh * inv, eps,
                                                                s0, s1, s2, grad, touched, loss_sum));
    }
    return check_launch(fn);
}

}  // namespace
}  // namespace plx

extern "C" int plx_tv_grad(const plx_grid *grid, int64_t cell_start, int64_t cell_count,
                           float lambda_sigma, float lambda_sh, float eps, float *grad,
                           uint8_t *touched, double *loss_sum, plx_stream stream) {
    return tv_launch(grid, cell_start, cell_count, lambda_sigma, lambda_sh, eps, grad, touched, loss_sum,
                     stream, false, "plx_tv_grad");
}

extern "C" int plx_bg_tv_grad(const plx_grid *bg_grid, int64_t cell_start, int64_t cell_count,
                              float lambda_sigma, float lambda_color, float eps, float *grad,
                              uint8_t *touched, double *loss_sum, plx_stream stream) {
    return tv_launch(bg_grid, cell_start, cell_count, lambda_sigma, lambda_color, eps, grad, touched,
                     loss_sum, stream, true, "plx_bg_tv_grad");
}
