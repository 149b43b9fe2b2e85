// render.hip -- differentiable volume rendering over the sparse voxel grid
// (Sec. 3.1-3.3, Eq. (1); supplement B.1) for gfx950.
//
// Work mapping: one ray per wave64 (four per 256-thread block).  The lanes
// form four rows of 16: row r < 3 holds the nine SH coefficients of colour
// channel r (lanes 16r .. 16r+8), row 3 holds the density (lane 48).  Every
// ray-level quantity is uniform over the wave, so corner ids, cells and
// sample masks live in scalar registers and all branches are uniform.
//
// SH factorisation.  The SH basis depends only on the ray direction, so the
// pre-activation colour of a sample is sum_c w_c (sum_l y_l k_{c,l}): the
// coefficients of a corner are projected on the ray's basis once, when the
// corner is loaded (one 4-byte load per lane and a 16-lane DPP reduction
// within each row), and each sample then interpolates four numbers per
// corner: row r of the wave interpolates channel r (r < 3) or density (r = 3).
// In the backward pass the gradient of a coefficient is y_l times the
// gradient of its channel's projected value, so the lanes accumulate one
// number per corner and multiply by y_l when the corner is flushed; the flush
// is one float atomic instruction per corner whose lanes cover one 128-byte
// record line.
//
// Exact empty-space skipping, two levels.  A sample whose lower-corner cell
// has no non-NULL corner reads only zeros: it changes neither colour nor
// transmittance and has no gradient.
//  - Brick level: every 8^3-cell brick stores its Chebyshev distance D (in
//    bricks) to the nearest brick with an occupied cell.  From a sample in a
//    brick with D > 0, every cell of the box of bricks within D-1 of it is
//    empty, so the ray jumps to the box's exit point along its own direction
//    (less a margin of 5% of a step, far above FP32 rounding of t and g).
//  - Cell level: near occupied bricks, 64 candidate samples are placed at a
//    time (one per lane) and tested against the cell bitmap; one ballot gives
//    the occupied ones, which are processed in order, each reading its cell
//    and interpolation weights from the lane that placed it.
// The corner ids and projected values of the current cell stay in registers
// while consecutive samples stay in one cell; a move to a face-adjacent cell
// keeps the 4 shared corners and loads only the other 4.
//
// Transmittance is exp(-tau) of the FP64 optical depth in both passes.
//
// Backward.  The ray is replayed from its last sample to its first.  With
// tau_after the optical depth after sample k (starting from the forward
// total), T_{k+1} = exp(-tau_after), T_k = exp(-(tau_after - sigma delta))
// and the rest of the ray R_k = sum_{j>k} w_j c_j + T_n bg is a running sum;
// dC/dsigma_k = delta (T_{k+1} c_k - R_k), dC/dc_k = w_k.  Corner gradients
// are accumulated in registers for as long as a voxel stays a corner of the
// current cell.  The fused training kernel keeps the list of non-empty
// 64-sample chunks found by its forward pass in LDS and replays exactly those
// in reverse.
#include <string.h>

#include <vector>

#include "plx_internal.hpp"

namespace plx {
namespace {

constexpr int kWave = 64;
constexpr int kThreads = 256;                    // 4 waves
constexpr int kRaysPerBlock = kThreads / kWave;  // 4
constexpr int kChunk = 64;                       // candidate samples per round (one per lane)
constexpr int kMaxChunks = 40;                   // chunk list entries per ray (fused kernel)
constexpr float kSkipMargin = 0.05f;             // in steps
constexpr int kSigmaLane = 48;                   // row 3, first lane

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
    uint8_t *touched;       // BWD, TRAIN
    double *loss_sum;       // TRAIN
    int64_t n_rays;
    float bg[3];
    float loss_scale;
    int n_blocks;
    int nb8;
};

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)uni((int)(uint32_t)u), hi = (uint32_t)uni((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int lane_i(int v, int i) { return __builtin_amdgcn_readlane(v, i); }
__device__ __forceinline__ float lane_f(float v, int i) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}

template <int CTRL> __device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Sum over the 16 lanes of each row, left in every lane of the row.  Each
// step adds a partner's value (lane^1, lane^2, the mirrored quad, the
// mirrored half-row); the pairing is symmetric and addition commutes, so
// every lane of a row ends with the same bits.
__device__ __forceinline__ float row_sum(float v) {
    v += dpp_f<0xB1>(v);   // quad_perm(1,0,3,2)
    v += dpp_f<0x4E>(v);   // quad_perm(2,3,0,1)
    v += dpp_f<0x141>(v);  // row_half_mirror
    v += dpp_f<0x140>(v);  // row_mirror
    return v;
}

// Role of a lane: its row, the record slot it reads and writes (-1: none) and
// the SH basis value of that slot's coefficient at the ray direction (1 for
// the density slot).
struct Lane {
    int L;
    int row;
    int slot;
    float y;
};

__device__ inline Lane lane_role(const float d[3]) {
    Lane l;
    l.L = threadIdx.x & (kWave - 1);
    l.row = l.L >> 4;
    const int j = l.L & 15;
    if (l.row < 3 && j < 9) {
        l.slot = 9 * l.row + j;
        l.y = sh_basis_at(j, d[0], d[1], d[2]);
    } else if (l.L == kSigmaLane) {
        l.slot = PLX_SLOT_SIGMA;
        l.y = 1.0f;
    } else {
        l.slot = -1;
        l.y = 0.0f;
    }
    return l;
}

// Slot s (0..26 or PLX_SLOT_SIGMA) of a record as one 32-bit load plus a
// branch-free conversion.
template <int DT> struct Slot;
template <> struct Slot<PLX_F32> {
    __device__ static inline uint32_t raw(const void *data, int64_t id, int s) {
        return reinterpret_cast<const uint32_t *>(static_cast<const char *>(data) +
                                                  id * (int64_t)kRecF32Bytes)[s];
    }
    __device__ static inline float cvt(uint32_t r, int) { return __uint_as_float(r); }
};
template <int DT> struct Slot16 {
    // the 32-bit word holding 16-bit slot s, or the FP32 density at byte 56
    __device__ static inline uint32_t raw(const void *data, int64_t id, int s) {
        const uint32_t *p = reinterpret_cast<const uint32_t *>(static_cast<const char *>(data) +
                                                               id * (int64_t)kRec16Bytes);
        return p[s == PLX_SLOT_SIGMA ? 14 : (s >> 1)];
    }
    __device__ static inline float cvt(uint32_t r, int s) {
        const uint32_t h = (s & 1) ? (r >> 16) : (r & 0xffffu);
        const float v = DT == PLX_BF16 ? bf16_to_f32(h) : f16_to_f32(h);
        return s == PLX_SLOT_SIGMA ? __uint_as_float(r) : v;
    }
};
template <> struct Slot<PLX_BF16> : Slot16<PLX_BF16> {};
template <> struct Slot<PLX_F16> : Slot16<PLX_F16> {};

// Uniform copy of a grid descriptor read from memory.
__device__ inline GridDev uniform_grid(const GridDev &s) {
    GridDev g;
    g.nx = uni(s.nx);
    g.ny = uni(s.ny);
    g.nz = uni(s.nz);
    g.bx = uni(s.bx);
    g.by = uni(s.by);
    g.bz = uni(s.bz);
    for (int a = 0; a < 3; ++a) {
        g.scale[a] = uni(s.scale[a]);
        g.offset[a] = uni(s.offset[a]);
    }
    g.step = uni(s.step);
    auto up = [](const void *p) {
        return reinterpret_cast<const void *>(uni64((int64_t)reinterpret_cast<uint64_t>(p)));
    };
    g.index = static_cast<const int32_t *>(up(s.index));
    g.data = up(s.data);
    g.occ = static_cast<const uint32_t *>(up(s.occ));
    g.bdist = static_cast<const uint8_t *>(up(s.bdist));
    g.n_vox = uni64(s.n_vox);
    return g;
}

// ------------------------------------------------------------ corner cache

// The current cell: corner ids (uniform) and, per lane, its row's projected
// value of each corner (channel r: sum_l y_l k_{c,9r+l}; row 3: density).
struct CornerCache {
    int cell[3];  // lower corner; cell[0] < 0 = empty cache
    int ids[8];
    float q[8];
};

__device__ inline int64_t corner_offset(const GridDev &g, int c) {
    return ((c >> 2) & 1) * ((int64_t)g.ny * g.nz) + ((c >> 1) & 1) * (int64_t)g.nz + (c & 1);
}

// Loads the corners of `mask` (bit c = corner c) of the cell cc.cell.
template <int DT>
__device__ __forceinline__ void load_corners(const GridDev &g, CornerCache &cc, const Lane &ln,
                                             unsigned mask) {
    const int64_t lin = cell_id(g, cc.cell);
    int mine = -1;
    if (ln.L < 8 && ((mask >> ln.L) & 1u)) mine = g.index[lin + corner_offset(g, ln.L)];
    uint32_t raw[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if ((mask >> c) & 1u) {
            cc.ids[c] = lane_i(mine, c);
            raw[c] = 0u;
            if (cc.ids[c] >= 0 && ln.slot >= 0) raw[c] = Slot<DT>::raw(g.data, cc.ids[c], ln.slot);
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if ((mask >> c) & 1u) {
            const float v = (cc.ids[c] >= 0 && ln.slot >= 0) ? Slot<DT>::cvt(raw[c], ln.slot) : 0.0f;
            cc.q[c] = row_sum(ln.y * v);
        }
    }
}

// Adds the accumulated gradients of the corners in `mask` to the FP32
// gradient records (one atomic instruction per corner line), marks those
// corners touched, and clears their accumulators.
__device__ __forceinline__ void flush(float *grad, uint8_t *touched, const CornerCache &cc,
                                      float acc[8], const Lane &ln, unsigned mask) {
    int tid = -1;  // lane 56 + c marks corner c
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!((mask >> c) & 1u)) continue;
        if (cc.ids[c] >= 0) {
            const float gv = ln.row < 3 ? ln.y * acc[c] : acc[c];
            if (ln.slot >= 0 && gv != 0.0f)
                unsafeAtomicAdd(grad + (int64_t)cc.ids[c] * PLX_REC_SLOTS + ln.slot, gv);
            tid = ln.L == 56 + c ? cc.ids[c] : tid;
        }
        acc[c] = 0.0f;
    }
    if (tid >= 0) touched[tid] = 1;
}

// Moves the cache along one axis (BIT 4 = x, 2 = y, 1 = z) by +1 (PLUS) or
// -1: the four shared corners change position, the other four are flushed
// (backward) and reloaded.
template <int DT, bool BWD, int BIT, bool PLUS>
__device__ __forceinline__ void shift_cell(const GridDev &g, CornerCache &cc, float acc[8],
                                           float *grad, uint8_t *touched, const Lane &ln) {
    // positions that receive a shared corner (their old corner leaves)
    unsigned keep = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (((c & BIT) != 0) == !PLUS) keep |= 1u << c;
    if (BWD) flush(grad, touched, cc, acc, ln, keep);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if ((keep >> c) & 1u) {
            cc.ids[c] = cc.ids[c ^ BIT];
            cc.q[c] = cc.q[c ^ BIT];
            if (BWD) {
                acc[c] = acc[c ^ BIT];
                acc[c ^ BIT] = 0.0f;
            }
        }
    }
    constexpr int a = BIT == 4 ? 0 : (BIT == 2 ? 1 : 2);
    cc.cell[a] += PLUS ? 1 : -1;
    load_corners<DT>(g, cc, ln, 0xffu & ~keep);
}

// Makes `cell` the cached cell.
template <int DT, bool BWD>
__device__ __forceinline__ void move_to(const GridDev &g, CornerCache &cc, const int cell[3],
                                        float acc[8], float *grad, uint8_t *touched,
                                        const Lane &ln) {
    const int dx = cell[0] - cc.cell[0], dy = cell[1] - cc.cell[1], dz = cell[2] - cc.cell[2];
    if (dx == 0 && dy == 0 && dz == 0) return;
    if (cc.cell[0] >= 0 && abs(dx) + abs(dy) + abs(dz) == 1) {
        if (dx == 1) shift_cell<DT, BWD, 4, true>(g, cc, acc, grad, touched, ln);
        else if (dx == -1) shift_cell<DT, BWD, 4, false>(g, cc, acc, grad, touched, ln);
        else if (dy == 1) shift_cell<DT, BWD, 2, true>(g, cc, acc, grad, touched, ln);
        else if (dy == -1) shift_cell<DT, BWD, 2, false>(g, cc, acc, grad, touched, ln);
        else if (dz == 1) shift_cell<DT, BWD, 1, true>(g, cc, acc, grad, touched, ln);
        else shift_cell<DT, BWD, 1, false>(g, cc, acc, grad, touched, ln);
        return;
    }
    if (BWD && cc.cell[0] >= 0) flush(grad, touched, cc, acc, ln, 0xffu);
    cc.cell[0] = cell[0];
    cc.cell[1] = cell[1];
    cc.cell[2] = cell[2];
    load_corners<DT>(g, cc, ln, 0xffu);
}

__device__ inline void corner_weights(const float f[3], float w[8]) {
    const float ax[2] = {1.0f - f[0], f[0]};
    const float ay[2] = {1.0f - f[1], f[1]};
    const float az[2] = {1.0f - f[2], f[2]};
#pragma unroll
    for (int c = 0; c < 8; ++c) w[c] = ax[(c >> 2) & 1] * ay[(c >> 1) & 1] * az[c & 1];
}

// ------------------------------------------------------------ samples

// Places the 64 candidate samples k0..k0+63 (sample k0+L in lane L).  With
// TEST, returns the uniform mask of those that exist and lie in an occupied
// cell.
template <bool TEST>
__device__ __forceinline__ uint64_t place_chunk(const GridDev &g, const RayGeom &r, int n, int k0,
                                                int L, Sample &s) {
    const int k = k0 + L;
    bool ne = false;
    s.cell[0] = s.cell[1] = s.cell[2] = 0;
    s.f[0] = s.f[1] = s.f[2] = 0.0f;
    s.delta = 0.0f;
    if (k >= 0 && k < n) {
        s = sample_at(g, r, k);
        if (TEST) ne = cell_occupied(g, cell_id(g, s.cell));
    }
    return TEST ? __ballot(ne) : 0ull;
}

// The sample placed in lane i, as uniform values.
struct USample {
    int cell[3];
    float w[8];
    float delta;
};

__device__ __forceinline__ USample take_sample(const Sample &s, int i) {
    USample u;
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u.cell[a] = lane_i(s.cell[a], i);
        f[a] = lane_f(s.f[a], i);
    }
    u.delta = lane_f(s.delta, i);
    corner_weights(f, u.w);
    return u;
}

// Brick-level skip.  Returns the distance D of the brick of sample k (0 when
// it has an occupied cell); for D > 0 also the number of further samples m
// (in the direction of travel) that certainly stay in the empty box of bricks
// within D-1 of it.
template <bool FORWARD>
__device__ __forceinline__ int brick_skip(const GridDev &g, const RayGeom &r, int k, int *m) {
    const Sample s = sample_at(g, r, k);
    const int b[3] = {s.cell[0] / PLX_BRICK, s.cell[1] / PLX_BRICK, s.cell[2] / PLX_BRICK};
    const int D = uni((int)g.bdist[((int64_t)b[0] * g.by + b[1]) * g.bz + b[2]]);
    if (D == 0) return 0;
    const int nb[3] = {g.bx, g.by, g.bz};
    const float t = r.t_near + (float)k * g.step;
    float t_edge = FORWARD ? __builtin_inff() : -__builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float dg = r.dg[a];
        if (dg == 0.0f) continue;
        // box faces on the grid boundary are never crossed by a sample
        const bool up = (dg > 0.0f) == FORWARD;
        const int bf = up ? b[a] + (D - 1) : b[a] - (D - 1);
        if (up ? bf >= nb[a] - 1 : bf <= 0) continue;
        const float face = (float)((up ? bf + 1 : bf) * PLX_BRICK);
        const float tf = (face - r.og[a]) / dg;
        t_edge = FORWARD ? fminf(t_edge, tf) : fmaxf(t_edge, tf);
    }
    const float span = FORWARD ? (t_edge - t) : (t - t_edge);
    float q = span / g.step - kSkipMargin;
    q = q < (float)kMaxSamples ? q : (float)kMaxSamples;
    *m = uni(q > 0.0f ? (int)q : 0);
    return D;
}

// Uniform ray: origin and direction of ray `ray` in every lane.
__device__ __forceinline__ void load_ray(const float *o_in, const float *d_in, int64_t ray,
                                         float o[3], float d[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = uni(o_in[3 * ray + i]);
        d[i] = uni(d_in[3 * ray + i]);
    }
}

// ------------------------------------------------------------ forward march

struct ChunkList {
    int *k0;
    unsigned long long *mask;
};

// Front-to-back march of one ray (Eq. (1)).  Returns in C the colour of the
// lane's row before the background is added (rows 0..2), and the optical
// depth in tau.  With RECORD, the non-empty chunks are appended to `list`
// (capacity kMaxChunks; *overflow is set when it runs out).
template <int DT, bool RECORD>
__device__ __forceinline__ void march_forward(const GridDev &g, const RayGeom &r, int n,
                                              const Lane &ln, CornerCache &cc, float &C,
                                              double &tau, ChunkList list, int &n_list,
                                              bool &overflow) {
    C = 0.0f;
    tau = 0.0;
    int k = 0;
    while (k < n) {
        int m;
        if (brick_skip<true>(g, r, k, &m)) {
            k += m + 1;
            continue;
        }
        Sample s;
        uint64_t mask = place_chunk<true>(g, r, n, k, ln.L, s);
        if (RECORD && mask) {
            if (n_list < kMaxChunks) {
                if (ln.L == 0) {
                    list.k0[n_list] = k;
                    list.mask[n_list] = mask;
                }
                ++n_list;
            } else {
                overflow = true;
            }
        }
        while (mask) {
            const int i = __builtin_ctzll(mask);
            mask &= mask - 1;
            const USample u = take_sample(s, i);
            move_to<DT, false>(g, cc, u.cell, nullptr, nullptr, nullptr, ln);
            float v = 0.0f;
#pragma unroll
            for (int c = 0; c < 8; ++c) v += u.w[c] * cc.q[c];
            const float sigma = fmaxf(lane_f(v, kSigmaLane), 0.0f);
            const float sd = sigma * u.delta;
            const float wk = expf(-(float)tau) * (-expm1f(-sd));
            C += wk * fmaxf(v, 0.0f);
            tau += (double)sd;
        }
        k += kChunk;
    }
}

// ------------------------------------------------------------------ kernel

template <int DT, int MODE>
__global__ __launch_bounds__(kThreads) void render_kernel(GridDev g, RenderArgs a) {
    constexpr bool FWD = MODE == MODE_FWD || MODE == MODE_TRAIN;
    constexpr bool BWD = MODE == MODE_BWD || MODE == MODE_TRAIN;
    constexpr int kList = MODE == MODE_TRAIN ? kRaysPerBlock * kMaxChunks : 1;
    __shared__ int list_k0[kList];
    __shared__ unsigned long long list_mask[kList];
    __shared__ double blk_loss;
    __shared__ unsigned blk_done;

    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    if (MODE == MODE_TRAIN) {
        if (threadIdx.x == 0) {
            blk_loss = 0.0;
            blk_done = 0u;
        }
        __syncthreads();
    }
    const int wid = uni((int)(threadIdx.x / kWave));
    const int64_t ray = (int64_t)blk * kRaysPerBlock + wid;
    if (ray >= a.n_rays) return;  // the whole wave

    float o[3], d[3];
    load_ray(a.rays_o, a.rays_d, ray, o, d);
    RayGeom r;
    const int n = ray_setup(g, o, d, r);
    const Lane ln = lane_role(d);

    CornerCache cc;
    cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
    float acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0f;

    // optical depth in FP64: transmittance is exp(-tau) in both passes, so
    // its error stays at one float rounding of tau instead of growing with the
    // number of samples
    double tau = 0.0;
    float gr[3] = {0.f, 0.f, 0.f};
    int n_list = 0;
    bool overflow = false;
    ChunkList list;
    list.k0 = list_k0 + (MODE == MODE_TRAIN ? wid * kMaxChunks : 0);
    list.mask = list_mask + (MODE == MODE_TRAIN ? wid * kMaxChunks : 0);

    // ------------------------------------------------------------ forward
    if (FWD) {
        float Crow;
        march_forward<DT, MODE == MODE_TRAIN>(g, r, n, ln, cc, Crow, tau, list, n_list, overflow);
        const float T_final = expf(-(float)tau);
        float C[3];
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) C[c3] = lane_f(Crow, 16 * c3) + T_final * a.bg[c3];
        if (ln.L == 0) {
            if (MODE == MODE_FWD || a.rgb_out) {
#pragma unroll
                for (int c3 = 0; c3 < 3; ++c3) a.rgb_out[3 * ray + c3] = C[c3];
            }
            if (MODE == MODE_FWD && a.tau_out) a.tau_out[ray] = (float)tau;
        }
        if (MODE == MODE_TRAIN) {
            float l2 = 0.0f;
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) {
                const float diff = C[c3] - uni(a.target[3 * ray + c3]);
                gr[c3] = 2.0f * a.loss_scale * diff;
                l2 += diff * diff;
            }
            // block sum in LDS; the block's last live wave adds it to the total
            if (ln.L == 0) {
                atomicAdd(&blk_loss, (double)a.loss_scale * (double)l2);
                __threadfence_block();
                const int64_t left = a.n_rays - (int64_t)blk * kRaysPerBlock;
                const unsigned live = left < kRaysPerBlock ? (unsigned)left : (unsigned)kRaysPerBlock;
                if (atomicAdd(&blk_done, 1u) == live - 1u) {
                    __threadfence_block();
                    unsafeAtomicAdd(a.loss_sum, atomicAdd(&blk_loss, 0.0));
                }
            }
        }
    }

    // ------------------------------------------------------------ backward
    if (BWD) {
        if (MODE == MODE_BWD) {
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) gr[c3] = uni(a.grad_rgb[3 * ray + c3]);
            tau = (double)uni(a.tau_in[ray]);
        }
        __builtin_amdgcn_wave_barrier();
        double tau_after = tau;
        float T_after = expf(-(float)tau_after);
        float gR = T_after * (gr[0] * a.bg[0] + gr[1] * a.bg[1] + gr[2] * a.bg[2]);
        // this row's colour gradient (0 on the density row)
        const float grow = ln.row == 0 ? gr[0] : (ln.row == 1 ? gr[1] : (ln.row == 2 ? gr[2] : 0.0f));
        // the cache may hold the forward pass's last cell: its corners have
        // nothing accumulated yet, which is what the backward expects
        const bool use_list = MODE == MODE_TRAIN && !overflow;
        int li = n_list - 1;  // list cursor (fused kernel)
        int k = n - 1;        // sample cursor (replay by traversal)
        while (use_list ? li >= 0 : k >= 0) {
            int k0;
            uint64_t mask;
            Sample s;
            if (use_list) {
                k0 = uni(list.k0[li]);
                const unsigned long long mk = list.mask[li];
                mask = ((uint64_t)(uint32_t)uni((int)(uint32_t)(mk >> 32)) << 32) |
                       (uint64_t)(uint32_t)uni((int)(uint32_t)mk);
                --li;
                place_chunk<false>(g, r, n, k0, ln.L, s);
            } else {
                int m;
                if (brick_skip<false>(g, r, k, &m)) {
                    k -= m + 1;
                    continue;
                }
                k0 = k - (kChunk - 1);
                mask = place_chunk<true>(g, r, n, k0, ln.L, s);
                k -= kChunk;
            }
            while (mask) {
                const int i = 63 - __builtin_clzll(mask);
                mask &= ~(1ull << i);
                const USample u = take_sample(s, i);
                move_to<DT, true>(g, cc, u.cell, acc, a.grad, a.touched, ln);
                float v = 0.0f;
#pragma unroll
                for (int c = 0; c < 8; ++c) v += u.w[c] * cc.q[c];
                const float sigma_pre = lane_f(v, kSigmaLane);
                const float sd = fmaxf(sigma_pre, 0.0f) * u.delta;
                const double tau_before = fmax(tau_after - (double)sd, 0.0);
                const float T_before = expf(-(float)tau_before);
                const float wk = T_before * (-expm1f(-sd));
                // d(colour . grad_rgb) / d(sigma) needs all three channels
                const float t = grow * fmaxf(v, 0.0f);
                const float gc = (lane_f(t, 0) + lane_f(t, 16)) + lane_f(t, 32);
                const float dsig = sigma_pre > 0.0f ? u.delta * (T_after * gc - gR) : 0.0f;
                const float g_row = ln.row < 3 ? (v > 0.0f ? wk * grow : 0.0f) : dsig;
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] += u.w[c] * g_row;
                gR += wk * gc;
                tau_after = tau_before;
                T_after = T_before;
            }
        }
        if (cc.cell[0] >= 0) flush(a.grad, a.touched, cc, acc, ln, 0xffu);
    }
}

// ------------------------------------------------------------------ novel views

// Pixel-centred pinhole ray of pixel (px, py) of a view, in FP64 with a fixed
// operation order (no contraction), rounded to FP32 once.
__device__ inline void camera_ray(const plx_view &v, int px, int py, float o[3], float d[3]) {
#pragma clang fp contract(off)
    const double x = ((double)px + 0.5 - 0.5 * (double)v.width) / v.focal;
    const double yv = -(((double)py + 0.5 - 0.5 * (double)v.height) / v.focal);
    const double z = -1.0;
    double dv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) dv[a] = v.c2w[4 * a + 0] * x + v.c2w[4 * a + 1] * yv + v.c2w[4 * a + 2] * z;
    const double nrm = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d[a] = (float)(dv[a] / nrm);
        o[a] = (float)v.c2w[4 * a + 3];
    }
}

constexpr int kTileW = 2, kTileH = 2;  // pixels per tile = rays per block

struct ViewsArgs {
    const GridDev *scenes;
    const plx_view *views;
    const int64_t *tile_start;  // [n_views + 1]
    unsigned long long *counter;
    int n_views;
    int64_t n_tiles;
    float bg[3];
    float *rgb_out;
};

// Persistent tile queue over all pixels of all views of the launch: each block
// takes the next 2x2-pixel tile, finds its view, generates the rays of its
// pixels (one per wave) and runs the same forward march as plx_render_fwd.  A
// pixel's colour depends only on its own ray and scene, never on the rest of
// the batch.
template <int DT>
__global__ __launch_bounds__(kThreads) void views_kernel(ViewsArgs a) {
    __shared__ long long tile_sh;
    const int wid = uni((int)(threadIdx.x / kWave));
    while (true) {
        if (threadIdx.x == 0) tile_sh = (long long)atomicAdd(a.counter, 1ull);
        __syncthreads();
        const int64_t tile = uni64(tile_sh);
        __syncthreads();
        if (tile >= a.n_tiles) break;
        int lo = 0, hi = a.n_views - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (uni64(a.tile_start[mid]) <= tile) lo = mid;
            else hi = mid - 1;
        }
        const plx_view &v = a.views[lo];
        const int width = uni(v.width), height = uni(v.height);
        const int64_t tl = tile - uni64(a.tile_start[lo]);
        const int tpr = (width + kTileW - 1) / kTileW;
        const int px = (int)(tl % tpr) * kTileW + (wid % kTileW);
        const int py = (int)(tl / tpr) * kTileH + (wid / kTileW);
        if (px < width && py < height) {
            const GridDev g = uniform_grid(a.scenes[uni(v.scene)]);
            float o[3], d[3];
            camera_ray(v, px, py, o, d);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                o[i] = uni(o[i]);
                d[i] = uni(d[i]);
            }
            RayGeom r;
            const int n = ray_setup(g, o, d, r);
            const Lane ln = lane_role(d);
            CornerCache cc;
            cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
            float Crow;
            double tau;
            int n_list = 0;
            bool overflow = false;
            ChunkList none = {nullptr, nullptr};
            march_forward<DT, false>(g, r, n, ln, cc, Crow, tau, none, n_list, overflow);
            const float T_final = expf(-(float)tau);
            float C[3];
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) C[c3] = lane_f(Crow, 16 * c3) + T_final * a.bg[c3];
            if (ln.L == 0) {
                float *out = a.rgb_out + 3 * (uni64(v.out_offset) + (int64_t)py * width + px);
#pragma unroll
                for (int c3 = 0; c3 < 3; ++c3) out[c3] = C[c3];
            }
        }
    }
}

struct ViewsLayout {
    int64_t counter, tile_start, scenes, views, bytes;
};

ViewsLayout views_layout(int32_t n_scenes, int32_t n_views) {
    auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
    ViewsLayout l;
    l.counter = 0;
    l.tile_start = 256;
    l.scenes = l.tile_start + up((int64_t)(n_views + 1) * (int64_t)sizeof(int64_t));
    l.views = l.scenes + up((int64_t)n_scenes * (int64_t)sizeof(GridDev));
    l.bytes = l.views + up((int64_t)n_views * (int64_t)sizeof(plx_view));
    return l;
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
        for (int k = 0; k < n; ++k) {
            const Sample s = sample_at(g, r, k);
            const int64_t lin = cell_id(g, s.cell);
            if (!cell_occupied(g, lin)) continue;
            ++n_occ;
            if (lin == last) continue;
            last = lin;
            for (int c = 0; c < 8; ++c) {
                const int64_t v = lin + corner_offset(g, c);
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
    if (n > ((int64_t)1 << 34)) return fail(PLX_EINVAL, "%s: n_rays too large", fn);
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
                   const float *tau_fwd, float *grad, uint8_t *touched, plx_stream stream) {
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
                     float *rgb_out, float *grad, uint8_t *touched, double *loss_sum,
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

int64_t plx_render_views_workspace(int32_t n_scenes, int32_t n_views) {
    if (n_scenes < 1 || n_views < 0) return 0;
    return views_layout(n_scenes, n_views).bytes;
}

int plx_render_views(const plx_grid *scenes, int32_t n_scenes, const plx_view *views,
                     int32_t n_views, const plx_render_opts *opts, float *rgb_out, void *workspace,
                     int64_t workspace_bytes, plx_stream stream) {
    const char *fn = "plx_render_views";
    if (!scenes || n_scenes < 1) return fail(PLX_EINVAL, "%s: need at least one scene", fn);
    if (n_views < 0) return fail(PLX_EINVAL, "%s: n_views < 0", fn);
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_views == 0) return PLX_OK;
    if (!views || !rgb_out || !workspace) return fail(PLX_EINVAL, "%s: NULL views/rgb_out/workspace", fn);
    const ViewsLayout lay = views_layout(n_scenes, n_views);
    if (workspace_bytes < lay.bytes)
        return fail(PLX_EINVAL, "%s: workspace of %lld bytes, need %lld", fn, (long long)workspace_bytes,
                    (long long)lay.bytes);
    const int32_t dt = scenes[0].sh_dtype;
    for (int32_t s = 0; s < n_scenes; ++s) {
        int rc = validate_grid(&scenes[s], true, fn);
        if (rc) return rc;
        if (scenes[s].sh_dtype != dt) return fail(PLX_EINVAL, "%s: scenes must share one sh_dtype", fn);
    }
    // host image of the workspace: counter, tile offsets, scene and view tables
    std::vector<unsigned char> img((size_t)lay.bytes, 0);
    int64_t *tile_start = reinterpret_cast<int64_t *>(img.data() + lay.tile_start);
    int64_t tiles = 0;
    for (int32_t i = 0; i < n_views; ++i) {
        const plx_view &v = views[i];
        if (v.scene < 0 || v.scene >= n_scenes) return fail(PLX_EINVAL, "%s: view %d: bad scene", fn, i);
        if (v.width < 1 || v.height < 1 || v.width > 65536 || v.height > 65536)
            return fail(PLX_EINVAL, "%s: view %d: bad size %dx%d", fn, i, v.width, v.height);
        if (!(v.focal > 0.0) || v.out_offset < 0)
            return fail(PLX_EINVAL, "%s: view %d: bad focal or out_offset", fn, i);
        tile_start[i] = tiles;
        tiles += (int64_t)((v.width + kTileW - 1) / kTileW) * ((v.height + kTileH - 1) / kTileH);
    }
    tile_start[n_views] = tiles;
    GridDev *sc = reinterpret_cast<GridDev *>(img.data() + lay.scenes);
    for (int32_t s = 0; s < n_scenes; ++s) sc[s] = to_dev(&scenes[s]);
    memcpy(img.data() + lay.views, views, sizeof(plx_view) * (size_t)n_views);
    hipStream_t s = as_stream(stream);
    PLX_CHECK_HIP(hipMemcpyAsync(workspace, img.data(), (size_t)lay.bytes, hipMemcpyHostToDevice, s), fn);
    // the host image is released on return: wait for the copy
    PLX_CHECK_HIP(hipStreamSynchronize(s), fn);
    char *ws = static_cast<char *>(workspace);
    ViewsArgs va;
    va.counter = reinterpret_cast<unsigned long long *>(ws + lay.counter);
    va.tile_start = reinterpret_cast<const int64_t *>(ws + lay.tile_start);
    va.scenes = reinterpret_cast<const GridDev *>(ws + lay.scenes);
    va.views = reinterpret_cast<const plx_view *>(ws + lay.views);
    va.n_views = n_views;
    va.n_tiles = tiles;
    va.rgb_out = rgb_out;
    for (int i = 0; i < 3; ++i) va.bg[i] = opts->background[i];
    const int64_t nblk = tiles < 4096 ? tiles : 4096;  // persistent: about 16 blocks per CU
    PLX_DISPATCH_DT(dt, DT, views_kernel<DT><<<(unsigned)nblk, kThreads, 0, s>>>(va));
    return check_launch(fn);
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
    if ((rc = count_set_bits(cell_mark, n_cells(grid->reso), &cells, s, fn))) return rc;
    if ((rc = count_set_bits(vox_mark, grid->n_vox, &vox, s, fn))) return rc;
    counts[2] = cells;
    counts[3] = vox;
    return PLX_OK;
}

}  // extern "C"
