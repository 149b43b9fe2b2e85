// render.hip -- differentiable volume rendering over the sparse voxel grid
// (Sec. 3.1-3.3, Eq. (1); supplement B.1) for gfx950.
//
// Work mapping: one ray per lane, 256 rays per block.  A heavily sampled
// ray is a long chain of dependent memory accesses (occupancy bits, index
// entries, voxel records), so the kernels keep as many rays in flight as the
// register file allows rather than spreading one ray over a wave.
//
// SH factorisation.  The SH basis depends only on the ray direction, so the
// pre-activation colour of a sample is sum_c w_c (sum_l y_l k_{c,l}): when a
// corner voxel is loaded its coefficients are projected on the ray's basis
// once, and each sample interpolates four numbers per corner (density and
// the three projected channels).  In the backward pass the gradient of a
// coefficient is y_l times the gradient of its channel's projected value,
// so a lane accumulates four numbers per corner.
//
// Exact empty-space skipping, two levels.  A sample whose lower-corner cell
// has no non-NULL corner reads only zeros: it changes neither colour nor
// transmittance and has no gradient.
//  - Brick level: every 8^3-cell brick stores its Chebyshev distance D (in
//    bricks) to the nearest brick with an occupied cell.  From a sample in a
//    brick with D > 0, every cell of the box of bricks within D-1 of it is
//    empty, so the ray jumps to the box's exit point along its own direction
//    (less a margin of 5% of a step, far above FP32 rounding of t and g).
//  - Cell level: near occupied bricks a lane tests 16 candidate samples at a
//    time against the cell bitmap (16 independent loads) and processes only
//    the occupied ones.
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
// current cell.  When it stops being one, the lane appends (voxel, four
// accumulated values, lane) to a queue in LDS; after every step of the
// replay the wave drains the queue two voxels at a time, 32 lanes per voxel,
// so that each voxel's 28 gradient values go out as one float atomic
// instruction covering its 128-byte gradient record (the access pattern for
// which the L2 float atomics are fastest).
//
// Priors (Sec. 3.7).  The Cauchy sparsity prior adds
// lambda_s 4 sigma / (1 + 2 sigma^2) to each sample's density gradient; the
// beta prior on T = T_final adds delta_k times one factor per ray,
// -T dL_b/dT, computed once from the ray's optical depth.  Both ride on the
// density slot of the same corner accumulators.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "plx_internal.hpp"

namespace plx {
namespace {

constexpr int kWave = 64;
constexpr int kThreads = 256;          // rays per block
constexpr int kWavesPerBlock = kThreads / kWave;
constexpr int kChunk = 16;             // candidate samples tested per round
constexpr int kQCap = 8 * kWave;       // queue entries per wave (8 corners per lane per step)
constexpr float kSkipMargin = 0.05f;   // in steps

enum { MODE_FWD = 0, MODE_BWD = 1, MODE_TRAIN = 2, MODE_MAXW = 3 };

// The optional sparsity (Cauchy) and beta priors of Sec. 3.7, as the gradient
// kernels see them.
struct Priors {
    float lambda_s;    // Cauchy weight (0 = off)
    float lambda_b;    // beta weight (0 = off)
    float eps;         // beta epsilon
    double *loss;      // [2] (L_s, L_b) ADDED, or NULL
};

// Background colour of a ray: its own when the call gives one per ray.
__device__ __forceinline__ void ray_background(const float *bg_rgb, const float bg[3], int64_t ray,
                                               float out[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = bg_rgb ? bg_rgb[3 * ray + c] : bg[c];
}

// Beta prior of one ray from its optical depth tau (FP64; 1 - T = -expm1(-tau)
// stays accurate for a nearly empty ray): returns dL_b/dsigma_k / delta_k =
// -T dL_b/dT, the factor of each of its samples' density gradient, and adds
// the ray's L_b to *loss.
__device__ inline float beta_factor(const Priors &p, double tau, double *loss) {
    const double T = exp(-tau), omT = -expm1(-tau), e = (double)p.eps;
    *loss += (double)p.lambda_b * (log(e + T) + log(e + omT));
    return (float)(-T * (double)p.lambda_b * (1.0 / (e + T) - 1.0 / (e + omT)));
}

// Cauchy prior at a sample with pre-activation density s > 0: the density
// gradient lambda_s 4 s / (1 + 2 s^2); log(1 + 2 s^2) goes to *ls.
__device__ __forceinline__ float cauchy_grad(const Priors &p, float s, float *ls) {
    if (p.lambda_s == 0.0f || !(s > 0.0f)) return 0.0f;
    *ls += log1pf(2.0f * s * s);
    return 4.0f * (p.lambda_s * s) / (1.0f + 2.0f * s * s);
}

// Adds a wave's prior losses to p.loss (one atomic per wave and term; the
// per-lane Cauchy sums are FP32, the wave sum FP64).
__device__ inline void add_prior_loss(const Priors &p, float ls_lane, double lb) {
    if (!p.loss) return;
    double ls = (double)ls_lane;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        ls += __shfl_xor(ls, m);
        lb += __shfl_xor(lb, m);
    }
    if ((threadIdx.x & 63) == 0) {
        if (ls != 0.0) unsafeAtomicAdd(p.loss, (double)p.lambda_s * ls);
        if (lb != 0.0) unsafeAtomicAdd(p.loss + 1, lb);
    }
}

// Arguments of the ray-order kernels of the stored-state calls (forward
// recording the samples, backward replaying them).
struct RenderArgs {
    const float *rays_o;
    const float *rays_d;
    const float *grad_rgb;  // BWD
    const float *tau_in;    // BWD
    float *rgb_out;         // FWD
    float *tau_out;         // FWD (optional)
    float *grad;            // BWD
    uint8_t *touched;       // BWD
    int *st_count;          // per-ray sample state (optional): occupied samples of each ray
    int *st_kidx;           // [n_rays][st_cap] their sample indices
    float4 *st_vals;        // [n_rays][st_cap] pre-activation density and projected colour
    int st_cap;
    int64_t n_rays;
    float bg[3];
    const float *bg_rgb;    // optional per-ray background colours [n_rays][3]
    float *grad_bg;         // BWD, optional: T_final dL/dC per ray [n_rays][3]
    Priors pri;
    int n_blocks;
    int nb8;
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Wave-uniform copies (readfirstlane) of values the compiler cannot prove
// uniform, so that they live in scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)uni((int)(uint32_t)u), hi = (uint32_t)uni((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T> __device__ __forceinline__ T *uni_ptr(T *p) {
    return reinterpret_cast<T *>(uni64((int64_t)reinterpret_cast<uintptr_t>(p)));
}

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
    g.index = uni_ptr(s.index);
    g.data = uni_ptr(s.data);
    g.occ = uni_ptr(s.occ);
    g.bdist = uni_ptr(s.bdist);
    g.n_vox = uni64(s.n_vox);
    return g;
}

// ------------------------------------------------------------ voxel records

// Density and the three colour channels projected on the ray's SH basis y.
struct Q4 {
    float s, r, g, b;
};

__device__ __forceinline__ Q4 q4_zero() { return Q4{0.0f, 0.0f, 0.0f, 0.0f}; }

template <int DT> struct Project;
template <> struct Project<PLX_F32> {
    // slots 0..27 as seven 16-byte loads, sigma (slot 28) as one 4-byte load
    __device__ static inline Q4 run(const void *data, int id, const float y[9]) {
        const float *rec = static_cast<const float *>(data) + (int64_t)id * PLX_REC_SLOTS;
        const float4 *p = reinterpret_cast<const float4 *>(rec);
        float v[28];
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const float4 t = p[i];
            v[4 * i] = t.x;
            v[4 * i + 1] = t.y;
            v[4 * i + 2] = t.z;
            v[4 * i + 3] = t.w;
        }
        Q4 q;
        q.s = rec[PLX_SLOT_SIGMA];
        q.r = 0.0f;
        q.g = 0.0f;
        q.b = 0.0f;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            q.r += y[l] * v[l];
            q.g += y[l] * v[9 + l];
            q.b += y[l] * v[18 + l];
        }
        return q;
    }
};
template <int DT> struct Project16 {
    // the 64-byte record as four 16-byte loads: 16-bit slot s in word s/2,
    // the FP32 density in word 14
    __device__ static inline float h2f(uint32_t h) {
        return DT == PLX_BF16 ? bf16_to_f32(h) : f16_to_f32(h);
    }
    __device__ static inline float slot(const uint32_t w[16], int s) {
        return h2f((s & 1) ? (w[s >> 1] >> 16) : (w[s >> 1] & 0xffffu));
    }
    __device__ static inline Q4 run(const void *data, int id, const float y[9]) {
        const uint4 *p = reinterpret_cast<const uint4 *>(static_cast<const char *>(data) +
                                                         (int64_t)id * kRec16Bytes);
        uint32_t w[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint4 t = p[i];
            w[4 * i] = t.x;
            w[4 * i + 1] = t.y;
            w[4 * i + 2] = t.z;
            w[4 * i + 3] = t.w;
        }
        Q4 q;
        q.s = __uint_as_float(w[14]);
        q.r = 0.0f;
        q.g = 0.0f;
        q.b = 0.0f;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            q.r += y[l] * slot(w, l);
            q.g += y[l] * slot(w, 9 + l);
            q.b += y[l] * slot(w, 18 + l);
        }
        return q;
    }
};
template <> struct Project<PLX_BF16> : Project16<PLX_BF16> {};
template <> struct Project<PLX_F16> : Project16<PLX_F16> {};

// ------------------------------------------------------------ flush queue

// The lane's current cell: corner ids and projected values.
struct CornerCache {
    int cell[3];  // lower corner; cell[0] < 0 = empty cache
    int ids[8];
    Q4 q[8];
};


// Per-wave queue of flushed corners in LDS (structure of arrays).
struct Queue {
    int *count;     // entries in use
    int *id;        // [kQCap] voxel id
    uint8_t *src;   // [kQCap] lane that flushed it (selects the SH basis)
    float4 *v;      // [kQCap] accumulated density, R, G, B gradients
    float *y;       // [64][9] SH basis of each lane's ray
};

__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Appends, for every active lane, its corners in `mask` (bit c = corner c)
// that are not NULL, with their accumulators.  One offset reservation per
// call: a lane's entries start at the sum of the counts of the active lanes
// below it (from the bit planes of the counts); only this wave uses the
// queue, and its LDS accesses are ordered.
__device__ __forceinline__ void push_corners(const Queue &qu, const CornerCache &cc,
                                             const Q4 acc[8], unsigned mask) {
    unsigned m = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (((mask >> c) & 1u) && cc.ids[c] >= 0) m |= 1u << c;
    const int cnt = __popc(m);
    int before = 0, total = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint64_t plane = __ballot((cnt >> b) & 1);
        before += lanes_below(plane) << b;
        total += __popcll(plane) << b;
    }
    if (total == 0) return;
    const uint64_t act = __ballot(1);
    const int leader = __builtin_ctzll(act);
    int base = 0;
    if (lane_id() == leader) {
        base = *qu.count;
        *qu.count = base + total;
    }
    base = __builtin_amdgcn_readlane(base, leader);
    int e = base + before;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if ((m >> c) & 1u) {
            qu.id[e] = cc.ids[c];
            qu.src[e] = (uint8_t)lane_id();
            qu.v[e] = make_float4(acc[c].s, acc[c].r, acc[c].g, acc[c].b);
            ++e;
        }
    }
}

// Sends every queued voxel's gradient to its FP32 record: lanes 0..31 take
// one entry and lanes 32..63 the next, lane L & 31 = record slot (0..26 SH,
// 28 density, 29 marks the voxel touched).  Called by the whole wave.  The
// LDS reads are unconditional (positions past the count are clamped into the
// queue and their values discarded), so the reads of a round overlap and
// the only branches are the ones around the stores.
__device__ __forceinline__ void drain(const Queue &qu, float *grad, uint8_t *touched) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int E = __builtin_amdgcn_readfirstlane(*qu.count);
    if (E == 0) return;
    const int L = lane_id();
    const int s = L & 31;
    const bool sh = s < PLX_NSH;
    const int ch = sh ? 1 + s / 9 : 0;  // v component: 0 density, 1..3 colour
    const int l = sh ? s % 9 : 0;
    const bool writes = sh || s == PLX_SLOT_SIGMA;
    const bool marks = s == PLX_SLOT_SIGMA + 1;
    float *gs = grad + s;
    const int half = L >> 5;
    // eight pairs of entries per round
    constexpr int U = 8;
    for (int b0 = 0; b0 < E; b0 += 2 * U) {
        const int e0 = b0 + half;
        int id[U], src[U];
        float a[U], yv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = min(e0 + 2 * u, kQCap - 1);
            id[u] = qu.id[e];
            src[u] = (int)qu.src[e] & (kWave - 1);
            a[u] = reinterpret_cast<const float *>(qu.v)[4 * e + ch];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) yv[u] = qu.y[src[u] * 9 + l];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = e0 + 2 * u < E;
            const float val = (ok && writes) ? (sh ? yv[u] : 1.0f) * a[u] : 0.0f;
            if (val != 0.0f) unsafeAtomicAdd(gs + (int64_t)id[u] * PLX_REC_SLOTS, val);
            if (ok && marks) touched[id[u]] = 1;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (L == 0) *qu.count = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------ corner cache


__device__ inline int64_t corner_offset(const GridDev &g, int c) {
    return ((c >> 2) & 1) * ((int64_t)g.ny * g.nz) + ((c >> 1) & 1) * (int64_t)g.nz + (c & 1);
}

template <class T> __device__ __forceinline__ void swap2(T &a, T &b) {
    const T t = a;
    a = b;
    b = t;
}

// Exchanges the corners at positions c and c ^ BIT (the two faces of the cell
// across axis BIT).  After a move by +-1 along that axis, the shared corners
// then sit at their new positions; the other four positions are reloaded.
template <int BIT, bool BWD>
__device__ __forceinline__ void swap_faces(CornerCache &cc, Q4 acc[8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (c & BIT) continue;
        swap2(cc.ids[c], cc.ids[c | BIT]);
        swap2(cc.q[c], cc.q[c | BIT]);
        if (BWD) swap2(acc[c], acc[c | BIT]);
    }
}

// Makes `cell` the lane's cached cell.  On a move to a face-adjacent cell the
// four shared corners change position (positions `keep` receive the corner
// at position ^ bit) and only the other four are loaded; on any other move
// all eight are.  Corners that stop being corners are flushed first
// (backward).  Without `project` only the corner ids are loaded (the replay
// of stored samples needs them for the scatter, not the values).
template <int DT, bool BWD>
__device__ __forceinline__ void move_to(const GridDev &g, CornerCache &cc, const int cell[3],
                                        Q4 acc[8], const Queue &qu, const float y[9],
                                        bool project = true) {
    const int dx = cell[0] - cc.cell[0], dy = cell[1] - cc.cell[1], dz = cell[2] - cc.cell[2];
    if (dx == 0 && dy == 0 && dz == 0) return;
    const bool had = cc.cell[0] >= 0;
    const bool adj = had && abs(dx) + abs(dy) + abs(dz) == 1;
    const int bit = dx != 0 ? 4 : (dy != 0 ? 2 : 1);
    const bool plus = dx + dy + dz > 0;
    unsigned keep = 0;
    if (adj) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (((c & bit) != 0) != plus) keep |= 1u << c;
    }
    if (BWD && had) {
        // corners leaving: those at `keep` positions (shift) or all (jump)
        push_corners(qu, cc, acc, adj ? keep : 0xffu);
    }
    if (adj) {
        if (bit == 4) swap_faces<4, BWD>(cc, acc);
        else if (bit == 2) swap_faces<2, BWD>(cc, acc);
        else swap_faces<1, BWD>(cc, acc);
    }
    cc.cell[0] = cell[0];
    cc.cell[1] = cell[1];
    cc.cell[2] = cell[2];
    const int64_t lin = cell_id(g, cc.cell);
    int nid[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) nid[c] = ((keep >> c) & 1u) ? cc.ids[c] : g.index[lin + corner_offset(g, c)];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!((keep >> c) & 1u)) {
            cc.ids[c] = nid[c];
            cc.q[c] = (project && nid[c] >= 0) ? Project<DT>::run(g.data, nid[c], y) : q4_zero();
            if (BWD) acc[c] = q4_zero();
        }
    }
}

__device__ inline void corner_weights(const float f[3], float w[8]) {
    const float ax[2] = {1.0f - f[0], f[0]};
    const float ay[2] = {1.0f - f[1], f[1]};
    const float az[2] = {1.0f - f[2], f[2]};
#pragma unroll
    for (int c = 0; c < 8; ++c) w[c] = ax[(c >> 2) & 1] * ay[(c >> 1) & 1] * az[c & 1];
}

// Interpolated (pre-activation) density and projected colour at weights w.
__device__ __forceinline__ Q4 interpolate(const CornerCache &cc, const float w[8]) {
    Q4 v = q4_zero();
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        v.s += w[c] * cc.q[c].s;
        v.r += w[c] * cc.q[c].r;
        v.g += w[c] * cc.q[c].g;
        v.b += w[c] * cc.q[c].b;
    }
    return v;
}

// ------------------------------------------------------------ sample cursor

// Occupancy of samples k0 .. k0+M-1 (bit i: sample k0+i exists and its cell
// is occupied); the M bitmap loads are independent.
// The loads are unconditional (indices outside [0, n) are clamped and their
// bits masked off afterwards): a load under a per-sample branch would be
// waited for inside that branch, serialising the 16 round trips.
template <int M = kChunk>
__device__ __forceinline__ uint32_t chunk_bits(const GridDev &g, const RayGeom &r, int n, int k0) {
    static_assert(M >= 1 && M < 32, "chunk size");
    constexpr uint32_t kFull = (1u << M) - 1u;
    const int k_max = n > 0 ? n - 1 : 0;
    uint32_t word[M];
    int bit[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        int k = k0 + i;
        k = k < 0 ? 0 : (k > k_max ? k_max : k);
        const Sample s = sample_at(g, r, k);
        const int64_t b = ((int64_t)(s.cell[0] >> 3) * g.by + (s.cell[1] >> 3)) * g.bz + (s.cell[2] >> 3);
        const int bb = ((s.cell[0] & 7) << 6) | ((s.cell[1] & 7) << 3) | (s.cell[2] & 7);
        word[i] = g.occ[b * 16 + (bb >> 5)];
        bit[i] = bb & 31;
    }
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < M; ++i) m |= ((word[i] >> bit[i]) & 1u) << i;
    // samples k0 + i inside [0, n)
    const int lo = k0 < 0 ? -k0 : 0;
    const int hi = n - k0;  // first i past the end
    uint32_t valid = hi <= 0 ? 0u : (hi >= M ? kFull : ((1u << hi) - 1u));
    valid &= lo >= M ? 0u : ((kFull << lo) & kFull);
    return m & valid;
}

// Number of further samples after sample k (in the direction of travel)
// that certainly stay inside the box of bricks within R of brick b, where
// sample k lies (at t = t_near + k*step): the box's exit parameter along the
// ray, less a margin of 5% of a step.
// Both walks over a ray's bricks (counting and emitting its segments) must
// cut identical segments, so this runs without FMA contraction like the
// sample recipe itself.
template <bool FORWARD>
__device__ __forceinline__ int samples_in_box(const GridDev &g, const RayGeom &r, int k,
                                              const int b[3], int R) {
#pragma clang fp contract(off)
    const int nb[3] = {g.bx, g.by, g.bz};
    const float t = r.t_near + (float)k * g.step;
    float t_edge = FORWARD ? __builtin_inff() : -__builtin_inff();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float dg = r.dg[a];
        if (dg == 0.0f) continue;
        // box faces on the grid boundary are never crossed by a sample
        const bool up = (dg > 0.0f) == FORWARD;
        const int bf = up ? b[a] + R : b[a] - R;
        if (up ? bf >= nb[a] - 1 : bf <= 0) continue;
        const float face = (float)((up ? bf + 1 : bf) * PLX_BRICK);
        const float tf = (face - r.og[a]) / dg;
        t_edge = FORWARD ? fminf(t_edge, tf) : fmaxf(t_edge, tf);
    }
    const float span = FORWARD ? (t_edge - t) : (t - t_edge);
    float q = span / g.step - kSkipMargin;
    q = q < (float)kMaxSamples ? q : (float)kMaxSamples;
    return q > 0.0f ? (int)q : 0;
}

__device__ __forceinline__ int64_t brick_id(const GridDev &g, const int b[3]) {
    return ((int64_t)b[0] * g.by + b[1]) * g.bz + b[2];
}

// Brick-level skip.  Returns the distance D of the brick of sample k (0 when
// it has an occupied cell); for D > 0 also the number of further samples m
// (in the direction of travel) that certainly stay in the empty box of bricks
// within D-1 of it.
template <bool FORWARD>
__device__ __forceinline__ int brick_skip(const GridDev &g, const RayGeom &r, int k, int *m) {
    const Sample s = sample_at(g, r, k);
    const int b[3] = {s.cell[0] / PLX_BRICK, s.cell[1] / PLX_BRICK, s.cell[2] / PLX_BRICK};
    const int D = g.bdist[brick_id(g, b)];
    if (D == 0) return 0;
    *m = samples_in_box<FORWARD>(g, r, k, b, D - 1);
    return D;
}

// Position in the ray's list of occupied samples.
struct Cursor {
    int k;          // next sample to examine
    int k0;         // first sample of the current chunk
    uint32_t mask;  // occupied samples of the chunk not yet returned
};

// Next occupied sample in increasing order, or -1 after the last one.
__device__ __forceinline__ int next_forward(const GridDev &g, const RayGeom &r, int n, Cursor &c) {
    while (c.mask == 0u) {
        if (c.k >= n) return -1;
        int m;
        if (brick_skip<true>(g, r, c.k, &m)) {
            c.k += m + 1;
            continue;
        }
        c.k0 = c.k;
        c.mask = chunk_bits(g, r, n, c.k);
        c.k += kChunk;
    }
    const int b = __builtin_ctz(c.mask);
    c.mask &= c.mask - 1u;
    return c.k0 + b;
}

// Next occupied sample in decreasing order, not below k_lo; -1 when done.
__device__ __forceinline__ int next_backward(const GridDev &g, const RayGeom &r, int n, int k_lo,
                                             Cursor &c) {
    while (c.mask == 0u) {
        if (c.k < k_lo) return -1;
        int m;
        if (brick_skip<false>(g, r, c.k, &m)) {
            c.k -= m + 1;
            continue;
        }
        c.k0 = c.k - (kChunk - 1);
        c.mask = chunk_bits(g, r, n, c.k0);
        if (c.k0 < k_lo) c.mask &= ~0u << (k_lo - c.k0);
        c.k -= kChunk;
    }
    const int b = 31 - __builtin_clz(c.mask);
    c.mask &= ~(1u << b);
    return c.k0 + b;
}

// ------------------------------------------------------------ forward march

// Front-to-back march of one ray (Eq. (1)).  Returns the colour before the
// background is added in C and the optical depth in tau.  With STORE, the
// first `cap` occupied samples (index and pre-activation values) go to
// kidx/vals and their total count to *count.
template <int DT, bool STORE = false>
__device__ __forceinline__ void march_forward(const GridDev &g, const RayGeom &r, int n,
                                              const float y[9], CornerCache &cc, float C[3],
                                              double &tau, int *count = nullptr, int *kidx = nullptr,
                                              float4 *vals = nullptr, int cap = 0) {
    C[0] = C[1] = C[2] = 0.0f;
    tau = 0.0;
    Cursor cur{0, 0, 0u};
    Q4 none[8];
    Queue noq{};
    int stored = 0;
    while (true) {
        const int k = next_forward(g, r, n, cur);
        if (k < 0) break;
        const Sample s = sample_at(g, r, k);
        move_to<DT, false>(g, cc, s.cell, none, noq, y);
        float w[8];
        corner_weights(s.f, w);
        const Q4 v = interpolate(cc, w);
        if (STORE) {
            if (stored < cap) {
                kidx[stored] = k;
                vals[stored] = make_float4(v.s, v.r, v.g, v.b);
            }
            ++stored;
        }
        const float sd = fmaxf(v.s, 0.0f) * s.delta;
        const float wk = expf(-(float)tau) * (-expm1f(-sd));
        C[0] += wk * fmaxf(v.r, 0.0f);
        C[1] += wk * fmaxf(v.g, 0.0f);
        C[2] += wk * fmaxf(v.b, 0.0f);
        tau += (double)sd;
    }
    if (STORE) *count = stored;
}

__device__ inline void sh_basis_all(const float d[3], float y[9]) {
#pragma unroll
    for (int l = 0; l < 9; ++l) y[l] = sh_basis_at(l, d[0], d[1], d[2]);
}

// ------------------------------------------------------------------ kernels

template <int DT, bool STORE>
__global__ __launch_bounds__(kThreads) void render_fwd_kernel(GridDev g, RenderArgs a) {
    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int64_t ray = (int64_t)blk * kThreads + threadIdx.x;
    if (ray >= a.n_rays) return;
    float o[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = a.rays_o[3 * ray + i];
        d[i] = a.rays_d[3 * ray + i];
    }
    RayGeom r;
    const int n = ray_setup(g, o, d, r);
    float y[9];
    sh_basis_all(d, y);
    CornerCache cc;
    cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
    float C[3];
    double tau;
    if (STORE) {
        const int64_t base = ray * a.st_cap;
        march_forward<DT, true>(g, r, n, y, cc, C, tau, a.st_count + ray,
                                a.st_kidx + base, a.st_vals + base, a.st_cap);
    } else {
        march_forward<DT>(g, r, n, y, cc, C, tau);
    }
    const float T_final = expf(-(float)tau);
    float bgc[3];
    ray_background(a.bg_rgb, a.bg, ray, bgc);
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) a.rgb_out[3 * ray + c3] = C[c3] + T_final * bgc[c3];
    if (a.tau_out) a.tau_out[ray] = (float)tau;
}

// Ray-order backward of the stored-state call.  Every lane of a block stays
// until its wave is done (the queue drains need all 64 lanes).  With STATE,
// a ray whose occupied samples were all stored by the forward pass replays
// them from the state (index loads only, no record gathers or
// interpolation); a ray with more than st_cap samples replays by traversal
// and recomputation.
template <int DT, bool STATE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
void render_bwd_kernel(GridDev g, RenderArgs a) {
    __shared__ int q_count[kWavesPerBlock];
    __shared__ int q_id[kWavesPerBlock * kQCap];
    __shared__ uint8_t q_src[kWavesPerBlock * kQCap];
    __shared__ float4 q_v[kWavesPerBlock * kQCap];
    __shared__ float q_y[kWavesPerBlock * kWave * 9];

    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int wid = threadIdx.x / kWave;
    const int L = lane_id();
    if (L == 0) q_count[wid] = 0;
    __syncthreads();
    Queue qu;
    qu.count = q_count + wid;
    qu.id = q_id + wid * kQCap;
    qu.src = q_src + wid * kQCap;
    qu.v = q_v + wid * kQCap;
    qu.y = q_y + wid * kWave * 9;

    const int64_t ray = (int64_t)blk * kThreads + threadIdx.x;
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
    // the lane's SH basis lives in the queue's table (read when a corner is
    // projected and when the wave drains the queue)
    float *y = qu.y + L * 9;
    sh_basis_all(d, y);

    CornerCache cc;
    cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
    Q4 acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = q4_zero();

    double tau = 0.0;
    float gr[3] = {0.f, 0.f, 0.f};
    const int k_lo = 0, k_hi = n - 1;
    float ls = 0.0f;
    double lb = 0.0;
    float gw = 0.0f;
    if (live) {
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) gr[c3] = a.grad_rgb[3 * ray + c3];
        tau = (double)a.tau_in[ray];
        if (a.pri.lambda_b != 0.0f) gw = beta_factor(a.pri, tau, &lb);
    }

    double tau_after = tau;
    float T_after = expf(-(float)tau_after);
    float bgc[3] = {0.f, 0.f, 0.f};
    if (live) {
        ray_background(a.bg_rgb, a.bg, ray, bgc);
        if (a.grad_bg) {
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) a.grad_bg[3 * ray + c3] = T_after * gr[c3];
        }
    }
    // g . R_k less the beta factor: dC/dsigma_k's delta (T_{k+1} g.c_k - g.R_k)
    // and the beta term's delta gw then share one running sum
    float gR = T_after * (gr[0] * bgc[0] + gr[1] * bgc[1] + gr[2] * bgc[2]) - gw;
    // the cache may hold the forward pass's last cell: its corners have
    // nothing accumulated yet, which is what the backward expects
    Cursor cur{k_hi, 0, 0u};
    bool active = live && n > 0 && k_lo <= k_hi;
    // stored samples of this ray (STATE): replayed from index j down to 0
    bool stored = false;
    int j = -1;
    int64_t st_base = 0;
    if (STATE && live) {
        const int cnt = a.st_count[ray];
        stored = cnt <= a.st_cap;
        j = cnt - 1;
        st_base = ray * a.st_cap;
        if (stored && cnt == 0) active = false;
    }
    while (__any(active)) {
        if (active) {
            int k;
            Q4 vs = q4_zero();
            if (STATE && stored) {
                k = -1;
                if (j >= 0) {
                    k = a.st_kidx[st_base + j];
                    const float4 t = a.st_vals[st_base + j];
                    vs = Q4{t.x, t.y, t.z, t.w};
                    --j;
                }
            } else {
                k = next_backward(g, r, n, k_lo, cur);
            }
            if (k < 0) {
                if (cc.cell[0] >= 0) push_corners(qu, cc, acc, 0xffu);
                active = false;
            } else {
                const Sample s = sample_at(g, r, k);
                move_to<DT, true>(g, cc, s.cell, acc, qu, y, !(STATE && stored));
                float w[8];
                corner_weights(s.f, w);
                const Q4 v = (STATE && stored) ? vs : interpolate(cc, w);
                const float sd = fmaxf(v.s, 0.0f) * s.delta;
                const double tau_before = fmax(tau_after - (double)sd, 0.0);
                const float T_before = expf(-(float)tau_before);
                const float wk = T_before * (-expm1f(-sd));
                const float gc = gr[0] * fmaxf(v.r, 0.0f) + gr[1] * fmaxf(v.g, 0.0f) +
                                 gr[2] * fmaxf(v.b, 0.0f);
                const float cs = cauchy_grad(a.pri, v.s, &ls);
                const float dsig = v.s > 0.0f ? s.delta * (T_after * gc - gR) + cs : 0.0f;
                const float g_r = v.r > 0.0f ? wk * gr[0] : 0.0f;
                const float g_g = v.g > 0.0f ? wk * gr[1] : 0.0f;
                const float g_b = v.b > 0.0f ? wk * gr[2] : 0.0f;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    acc[c].s += w[c] * dsig;
                    acc[c].r += w[c] * g_r;
                    acc[c].g += w[c] * g_g;
                    acc[c].b += w[c] * g_b;
                }
                gR += wk * gc;
                tau_after = tau_before;
                T_after = T_before;
            }
        }
        drain(qu, a.grad, a.touched);
    }
    add_prior_loss(a.pri, ls, lb);
}

// ------------------------------------------------------------ brick-binned training
//
// plx_render_fwd, plx_render_bwd and plx_render_train run the batch in brick
// order.  Rays sampled from many
// cameras share few voxels with their neighbours in the batch, so a ray-order
// pass fetches every voxel record (and read-modify-writes every gradient
// line) about as often as rays cross it.  Here each ray is cut into segments,
// one per 8^3-cell brick with occupied cells that its samples pass through
// (a ray crosses a brick at most once: cell indices are monotone along it);
// the segments are sorted by brick, and the forward and backward passes run
// one lane per segment in that order, so the lanes of a wave read and update
// the same few hundred voxels.  Per ray, the segment results compose exactly
// as the samples do: the colour is sum_s T_in(s) C_s + T_n bg with
// T_in(s) = exp(-sum_{s'<s} tau_s'), and the backward replay of a segment
// starts from the optical depth after it and the radiance the ray collects
// after it (g . R), so every sample sees the same T_k, w_k and R_k.
//
// The lanes of a wave march in step, so a wave takes as many trips as its
// longest segment.  Inside a brick the segments are therefore ordered by
// length class (the segment's number of samples in steps of kLenStep): the
// bins are keyed by (brick, class).  A wave's segments then have closer
// lengths while the order stays by brick (ordering by class first, across
// bricks, evens the lengths out further but loses more to the scattered
// record reads than it gains).

//
// The bricks themselves are ordered by tiles of kTile^3 bricks (tiles in
// storage order, bricks inside a tile in storage order), so that the
// segments of consecutive waves stay within a compact block of the grid
// rather than a row of bricks along z.

constexpr int kLenClasses = 8;
constexpr int kLenStep = 4;
constexpr int kTile = 4;
constexpr int kBrickCells = PLX_BRICK * PLX_BRICK * PLX_BRICK;           // 512
constexpr int kBrickVox = (PLX_BRICK + 1) * (PLX_BRICK + 1) * (PLX_BRICK + 1);  // 729 corner voxels

inline int tiles_along(int bricks) { return (bricks + kTile - 1) / kTile; }
// Number of (brick, class) bins: brick order positions times classes.
inline int64_t n_bins(const GridDev &g) {
    return (int64_t)tiles_along(g.bx) * tiles_along(g.by) * tiles_along(g.bz) * (kTile * kTile * kTile) *
           kLenClasses;
}

// Position of brick b in the binning order.
__device__ __forceinline__ int64_t brick_order(const GridDev &g, const int b[3]) {
    const int nty = (g.by + kTile - 1) / kTile, ntz = (g.bz + kTile - 1) / kTile;
    const int64_t tile = ((int64_t)(b[0] / kTile) * nty + b[1] / kTile) * ntz + b[2] / kTile;
    return tile * (kTile * kTile * kTile) + ((b[0] % kTile) * kTile + b[1] % kTile) * kTile + b[2] % kTile;
}

__device__ __forceinline__ int64_t seg_bin(int64_t order, int k0, int k1) {
    const int c = min((k1 - k0) / kLenStep, kLenClasses - 1);
    return order * kLenClasses + c;
}

constexpr int kScanT = 256, kScanI = 16, kScanTile = kScanT * kScanI;

// Exclusive block-wide scan of one int64 per thread; *total gets the sum.
template <int NT = kScanT>
__device__ int64_t block_scan_excl(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[NT / kWave];
    const int L = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (L >= o) x += y;
    }
    if (L == kWave - 1) wsum[w] = x;
    __syncthreads();
    int64_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) {
        if (i < w) before += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

// The counts are c[0], c[stride], c[2*stride], ... (stride 2 reads one half
// of an array of 64-bit counter pairs).
__global__ __launch_bounds__(kScanT) void count_sum_kernel(const unsigned *c, int64_t n, int stride,
                                                           int64_t *bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanI;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanI; ++i)
        if (base + i < n) s += c[(base + i) * stride];
    int64_t tot;
    block_scan_excl(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanT) void block_offsets_kernel(const int64_t *bsum, int64_t nb,
                                                               int64_t *boff) {
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanT) {
        const int64_t b = b0 + threadIdx.x;
        int64_t tot;
        const int64_t ex = block_scan_excl(b < nb ? bsum[b] : 0, &tot);
        if (b < nb) boff[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) boff[nb] = carry;
}

// out[i] = sum of c[0..i), out[n] = total.
__global__ __launch_bounds__(kScanT) void count_scan_kernel(const unsigned *c, int64_t n, int stride,
                                                            const int64_t *boff, int64_t *out) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanI;
    unsigned v[kScanI];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanI; ++i) {
        v[i] = base + i < n ? c[(base + i) * stride] : 0u;
        s += v[i];
    }
    int64_t tot;
    int64_t r = boff[blockIdx.x] + block_scan_excl(s, &tot);
#pragma unroll
    for (int i = 0; i < kScanI; ++i) {
        if (base + i < n) out[base + i] = r;
        r += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = boff[gridDim.x];
}

__global__ void zero_u32_kernel(unsigned *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// One occupied sample of the sample buffer, as the forward pass leaves it:
// its position in its cell, its sample index and cell, and the interpolated
// (pre-activation) density and projected colour.
struct SampleRec {
    float4 pos;   // f[0], f[1], f[2], (k << 9 | cell x*64 + y*8 + z) as integer bits
    float4 val;   // sigma, r, g, b
};

struct BinArgs {
    const float *rays_o;
    const float *rays_d;
    const float *target;    // TRAIN
    const float *grad_rgb;  // BWD
    float *tau_out;         // FWD (optional)
    float *rgb_out;
    double *loss_sum;
    float *grad;
    uint8_t *touched;
    int64_t n_rays;
    int64_t n_seg;
    float bg[3];
    const float *bg_rgb;    // optional per-ray background colours [n_rays][3]
    float *grad_bg;         // TRAIN/BWD, optional: T_final dL/dC per ray [n_rays][3]
    float loss_scale;
    int n_blocks;  // blocks of the launch at hand (rays or segments)
    int nb8;
    unsigned *nseg;      // [n_rays] segments of each ray
    int64_t *seg_off;    // [n_rays + 1] first ray-major slot of each ray
    unsigned *bcount;    // [n_bins] segments in each (length class, brick) bin
    unsigned *bcursor;   // [n_bins] placement cursors
    int64_t *boff;       // [n_bins + 1] first bin-major position of each bin
    int4 *bseg;          // [n_seg] bin-major: ray, first sample, last sample, ray-major slot
    double *tau_seg;     // [n_seg] ray-major: optical depth of the segment
    float4 *c_seg;       // [n_seg] ray-major: colour the segment adds (before T_in)
    double *tau_in;      // [n_seg] ray-major: optical depth before the segment
    float *gr_after;     // [n_seg] ray-major: g . (radiance collected after the segment)
    float4 *g_ray;       // [n_rays] dL/dC of each ray; w: beta factor of its samples
    unsigned *status;    // set to 1 when the emitting walk disagrees with the counting walk
    const int64_t *n_seg_dev;  // when set, the segment count is read here instead of n_seg
    void **events;       // optional hipEvent_t[4] recorded between the render kernels
    int64_t seg_cap;     // segment records the segment buffer holds
    // per-bin sample counts and the recorded backward (NULL when the bins
    // carry no sample buffer)
    unsigned long long *bcnt64;  // [n_bins] segments (low half) and sample slots (high half) per bin
    unsigned long long *bcur64;  // [n_bins] segment and sample placement cursors, packed the same way
    int64_t *bsoff;      // [n_bins + 1] first sample slot of each bin
    unsigned *blist;     // [n_brick] binning-order positions of the bricks with segments
    unsigned *nbrick;    // device count of blist entries
    int64_t n_brick;
    int64_t *soff;       // [n_seg] bin-major: first sample slot of each segment
    int *nocc;           // [n_seg] bin-major: occupied samples the replay recorded
    SampleRec *srec;     // [samp_cap] sample records
    int64_t samp_cap;
    Priors pri;
    float *wmax;         // MAXW: [M] per-voxel maximum sample weight
};

// Number of segments of the call: the host's count, or the device copy when
// the launch was sized by a bound instead.
__device__ __forceinline__ int64_t seg_count_of(const BinArgs &a) {
    return a.n_seg_dev ? min(*a.n_seg_dev, a.n_seg) : a.n_seg;
}

// A segment record with its ray and slot inside the call's arrays.  The emit
// walk repeats the count walk exactly, so every position holds a valid
// record; the check keeps a record that is not (a disagreement, which the
// emit kernel reports in the status word) from indexing outside the arrays.
__device__ __forceinline__ bool seg_valid(const BinArgs &a, const int4 &sg, int64_t n_seg) {
    return (uint64_t)(int64_t)sg.x < (uint64_t)a.n_rays && (uint64_t)(int64_t)sg.w < (uint64_t)n_seg;
}

__device__ __forceinline__ void load_ray_lane(const BinArgs &a, int64_t ray, float o[3], float d[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = a.rays_o[3 * ray + i];
        d[i] = a.rays_d[3 * ray + i];
    }
}

// Calls f(brick order position, first sample, last sample) for every brick
// with an occupied cell that the ray's samples enter, in ray order; boxes of
// empty bricks are skipped with the distance field, and inside a brick only
// the samples near its exit face are placed.
template <class F>
__device__ __forceinline__ void walk_bricks(const GridDev &g, const RayGeom &r, int n, F &&f) {
    int k = 0;
    while (k < n) {
        const Sample s = sample_at(g, r, k);
        const int b[3] = {s.cell[0] / PLX_BRICK, s.cell[1] / PLX_BRICK, s.cell[2] / PLX_BRICK};
        const int64_t bid = brick_id(g, b);
        const int D = g.bdist[bid];
        const int m = samples_in_box<true>(g, r, k, b, D > 0 ? D - 1 : 0);
        if (D > 0) {
            k += m + 1;
            continue;
        }
        int ke = m < n - 1 - k ? k + m : n - 1;
        while (ke + 1 < n) {
            const Sample s2 = sample_at(g, r, ke + 1);
            if (s2.cell[0] / PLX_BRICK != b[0] || s2.cell[1] / PLX_BRICK != b[1] ||
                s2.cell[2] / PLX_BRICK != b[2])
                break;
            ++ke;
        }
        f(brick_order(g, b), k, ke);
        k = ke + 1;
    }
}

__global__ __launch_bounds__(kThreads) void seg_count_kernel(GridDev g, BinArgs a) {
    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int64_t ray = (int64_t)blk * kThreads + threadIdx.x;
    if (ray >= a.n_rays) return;
    float o[3], d[3];
    load_ray_lane(a, ray, o, d);
    RayGeom r;
    const int n = ray_setup(g, o, d, r);
    unsigned cnt = 0;
    walk_bricks(g, r, n, [&](int64_t bid, int k0, int k1) {
        ++cnt;
        const int64_t bin = seg_bin(bid, k0, k1);
        if (a.bcnt64) atomicAdd(a.bcnt64 + bin, 1ull | ((unsigned long long)(k1 - k0 + 1) << 32));
        else atomicAdd(a.bcount + bin, 1u);
    });
    a.nseg[ray] = cnt;
}

__global__ __launch_bounds__(kThreads) void seg_emit_kernel(GridDev g, BinArgs a) {
    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int64_t ray = (int64_t)blk * kThreads + threadIdx.x;
    if (ray >= a.n_rays) return;
    float o[3], d[3];
    load_ray_lane(a, ray, o, d);
    RayGeom r;
    const int n = ray_setup(g, o, d, r);
    int64_t slot = a.seg_off[ray];
    const int64_t slot_end = a.seg_off[ray + 1];
    bool bad = false;
    walk_bricks(g, r, n, [&](int64_t bid, int k0, int k1) {
        const int64_t bin = seg_bin(bid, k0, k1);
        const unsigned len = (unsigned)(k1 - k0 + 1);
        // one cursor update gives the segment's position and (with a sample
        // buffer) its first sample slot
        unsigned long long cur = 0;
        if (a.bcur64) cur = atomicAdd(a.bcur64 + bin, 1ull | ((unsigned long long)len << 32));
        const int64_t pos = a.boff[bin] + (a.bcur64 ? (int64_t)(unsigned)cur : (int64_t)atomicAdd(a.bcursor + bin, 1u));
        // positions and slots stay inside the ranges the count reserved
        // and inside the segment buffer
        if (pos < a.boff[bin + 1] && slot < slot_end && pos < a.seg_cap && slot < a.seg_cap) {
            a.bseg[pos] = make_int4((int)ray, k0, k1, (int)slot);
            if (a.soff) {
                // the segment's sample slots, inside its bin's and the buffer's
                const int64_t sp = a.bsoff[bin] + (int64_t)(cur >> 32);
                const bool fits = sp + len <= a.bsoff[bin + 1] && sp + len <= a.samp_cap;
                a.soff[pos] = fits ? sp : -1;
                bad |= !fits;
            }
        } else {
            bad = true;
        }
        ++slot;
    });
    if (bad || slot != slot_end) *a.status = 1u;
}

// Appends the binning-order position of every brick with segments to
// a.blist (one counter update per wave; the order across waves is free).
__global__ __launch_bounds__(kThreads) void brick_list_kernel(BinArgs a, int64_t n_bricks) {
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool has = j < n_bricks && a.boff[(j + 1) * kLenClasses] > a.boff[j * kLenClasses];
    const uint64_t m = __ballot(has);
    if (m == 0) return;
    unsigned base = 0;
    if (lane_id() == 0) base = atomicAdd(a.nbrick, (unsigned)__popcll(m));
    base = __shfl(base, 0);
    if (has) a.blist[base + lanes_below(m)] = (unsigned)j;
}

// Occupied samples of [k_lo, k_hi] in increasing / decreasing order.
struct SpanCursor {
    int k;          // next sample to examine
    int k0;         // first sample of the current chunk
    uint32_t mask;  // occupied samples of the chunk not yet returned
};

__device__ __forceinline__ int span_next_up(const GridDev &g, const RayGeom &r, int n, int k_hi,
                                            SpanCursor &c) {
    while (c.mask == 0u) {
        if (c.k > k_hi) return -1;
        c.k0 = c.k;
        c.mask = chunk_bits(g, r, n, c.k);
        if (k_hi - c.k < kChunk - 1) c.mask &= (2u << (k_hi - c.k)) - 1u;
        c.k += kChunk;
    }
    const int b = __builtin_ctz(c.mask);
    c.mask &= c.mask - 1u;
    return c.k0 + b;
}

__device__ __forceinline__ int span_next_down(const GridDev &g, const RayGeom &r, int n, int k_lo,
                                              SpanCursor &c) {
    while (c.mask == 0u) {
        if (c.k < k_lo) return -1;
        c.k0 = c.k - (kChunk - 1);
        c.mask = chunk_bits(g, r, n, c.k0);
        if (c.k0 < k_lo) c.mask &= ~0u << (k_lo - c.k0);
        c.k -= kChunk;
    }
    const int b = 31 - __builtin_clz(c.mask);
    c.mask &= ~(1u << b);
    return c.k0 + b;
}

// Forward over one segment (transmittance relative to its start).  REC
// (the training and backward calls with a sample buffer) also stores every
// occupied sample's position in its cell, cell, sample index and
// interpolated values, in the segment's slots of the sample buffer.
template <int DT, bool REC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void seg_fwd_kernel(GridDev g, BinArgs a) {
    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    const int64_t n_seg = seg_count_of(a);
    if (i >= n_seg) return;
    const int4 sg = a.bseg[i];
    if (!seg_valid(a, sg, n_seg)) return;
    float o[3], d[3];
    load_ray_lane(a, sg.x, o, d);
    RayGeom r;
    const int n = ray_setup(g, o, d, r);
    float y[9];
    sh_basis_all(d, y);
    CornerCache cc;
    cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
    Q4 none[8];
    Queue noq{};
    SpanCursor cur{sg.y, 0, 0u};
    double tau = 0.0;
    float C[3] = {0.0f, 0.0f, 0.0f};
    int64_t base = 0, room = 0;
    if (REC) {
        base = a.soff[i];
        room = (int64_t)sg.z - sg.y + 1;  // the slots the count reserved
        if (base < 0 || base + room > a.samp_cap) room = 0;
    }
    int j = 0;
    while (true) {
        const int k = span_next_up(g, r, n, sg.z, cur);
        if (k < 0) break;
        const Sample s = sample_at(g, r, k);
        move_to<DT, false>(g, cc, s.cell, none, noq, y);
        float w[8];
        corner_weights(s.f, w);
        const Q4 v = interpolate(cc, w);
        if (REC && j < room) {
            const int code = (k << 9) | ((s.cell[0] & (PLX_BRICK - 1)) << 6) |
                             ((s.cell[1] & (PLX_BRICK - 1)) << 3) | (s.cell[2] & (PLX_BRICK - 1));
            SampleRec *rec = a.srec + base + j;
            rec->pos = make_float4(s.f[0], s.f[1], s.f[2], __int_as_float(code));
            rec->val = make_float4(v.s, v.r, v.g, v.b);
        }
        ++j;
        const float sd = fmaxf(v.s, 0.0f) * s.delta;
        const float wk = expf(-(float)tau) * (-expm1f(-sd));
        C[0] += wk * fmaxf(v.r, 0.0f);
        C[1] += wk * fmaxf(v.g, 0.0f);
        C[2] += wk * fmaxf(v.b, 0.0f);
        tau += (double)sd;
    }
    a.tau_seg[sg.w] = tau;
    a.c_seg[sg.w] = make_float4(C[0], C[1], C[2], 0.0f);
    if (REC) a.nocc[i] = (int)min((int64_t)j, room);
}

// ------------------------------------------------------------ brick-staged forward
//
// The segments of one brick read the same (at most 9^3) corner records, and
// at the training workload about 240 bricks are in flight per XCD at once,
// several times what its 4 MB L2 holds, so the lane-per-segment forward
// fetches each record from HBM several times.  The staged forward gives each
// brick with segments one workgroup: the brick's corner records are loaded
// once, coalesced, into LDS, and the workgroup's lanes march the brick's
// segments (one lane each) with the corner fetches served from LDS.  The
// arithmetic is that of seg_fwd.  It serves the forward renders of the
// 16-bit storage types, and their recording forward where bricks hold few
// segments (with many, the sample-parallel one below); FP32 records need
// 82 KB of LDS per brick, which leaves one workgroup (about two busy waves)
// per CU, and there the lane-per-segment kernel wins.

// 16-byte words of a staged record: FP32 slots 0..26 and the density in
// word 6's last float (28 floats); the 64-byte 16-bit record as stored.
template <int DT> struct StagedRec {
    static constexpr int kWords = DT == PLX_F32 ? 7 : 4;
};

template <int DT>
__device__ __forceinline__ Q4 project_staged(const uint4 *w4, const float y[9]) {
    if constexpr (DT == PLX_F32) {
        float v[28];
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const uint4 t = w4[i];
            v[4 * i] = __uint_as_float(t.x);
            v[4 * i + 1] = __uint_as_float(t.y);
            v[4 * i + 2] = __uint_as_float(t.z);
            v[4 * i + 3] = __uint_as_float(t.w);
        }
        Q4 q;
        q.s = v[27];
        q.r = 0.0f;
        q.g = 0.0f;
        q.b = 0.0f;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            q.r += y[l] * v[l];
            q.g += y[l] * v[9 + l];
            q.b += y[l] * v[18 + l];
        }
        return q;
    } else {
        uint32_t w[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint4 t = w4[i];
            w[4 * i] = t.x;
            w[4 * i + 1] = t.y;
            w[4 * i + 2] = t.z;
            w[4 * i + 3] = t.w;
        }
        Q4 q;
        q.s = __uint_as_float(w[14]);
        q.r = 0.0f;
        q.g = 0.0f;
        q.b = 0.0f;
#pragma unroll
        for (int l = 0; l < 9; ++l) {
            q.r += y[l] * Project16<DT>::slot(w, l);
            q.g += y[l] * Project16<DT>::slot(w, 9 + l);
            q.b += y[l] * Project16<DT>::slot(w, 18 + l);
        }
        return q;
    }
}

// move_to of the staged forward: cc.ids hold brick-local lattice positions
// (x*81 + y*9 + z) of non-NULL corners, -1 for NULL ones.
template <int DT>
__device__ __forceinline__ void move_staged(CornerCache &cc, const int cell[3], const int b0[3],
                                            const uint4 *s_rec, const int *s_id, const float y[9]) {
    const int dx = cell[0] - cc.cell[0], dy = cell[1] - cc.cell[1], dz = cell[2] - cc.cell[2];
    if (dx == 0 && dy == 0 && dz == 0) return;
    const bool had = cc.cell[0] >= 0;
    const bool adj = had && abs(dx) + abs(dy) + abs(dz) == 1;
    const int bit = dx != 0 ? 4 : (dy != 0 ? 2 : 1);
    const bool plus = dx + dy + dz > 0;
    unsigned keep = 0;
    if (adj) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (((c & bit) != 0) != plus) keep |= 1u << c;
        Q4 unused[8];
        if (bit == 4) swap_faces<4, false>(cc, unused);
        else if (bit == 2) swap_faces<2, false>(cc, unused);
        else swap_faces<1, false>(cc, unused);
    }
    cc.cell[0] = cell[0];
    cc.cell[1] = cell[1];
    cc.cell[2] = cell[2];
    const int lx = cell[0] - b0[0], ly = cell[1] - b0[1], lz = cell[2] - b0[2];
    const bool inside = (unsigned)lx < PLX_BRICK && (unsigned)ly < PLX_BRICK && (unsigned)lz < PLX_BRICK;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!((keep >> c) & 1u)) {
            const int p = (lx + ((c >> 2) & 1)) * 81 + (ly + ((c >> 1) & 1)) * 9 + (lz + (c & 1));
            const bool has = inside && s_id[p] >= 0;
            cc.ids[c] = has ? p : -1;
            cc.q[c] = has ? project_staged<DT>(s_rec + p * StagedRec<DT>::kWords, y) : q4_zero();
        }
    }
}

template <int DT, bool REC>
__global__ __launch_bounds__(kThreads) void seg_fwd_brick_kernel(GridDev g, BinArgs a) {
    constexpr int W = StagedRec<DT>::kWords;
    __shared__ uint4 s_rec[kBrickVox * W];
    __shared__ int s_id[kBrickVox];
    if (blockIdx.x >= (unsigned)a.n_brick) return;
    const int t = threadIdx.x;
    const int64_t jo = a.blist[blockIdx.x];
    const int nty = (g.by + kTile - 1) / kTile, ntz = (g.bz + kTile - 1) / kTile;
    const int64_t tile = jo / (kTile * kTile * kTile);
    const int in = (int)(jo % (kTile * kTile * kTile));
    const int b0[3] = {((int)(tile / ((int64_t)nty * ntz)) * kTile + in / (kTile * kTile)) * PLX_BRICK,
                       ((int)((tile / ntz) % nty) * kTile + (in / kTile) % kTile) * PLX_BRICK,
                       ((int)(tile % ntz) * kTile + in % kTile) * PLX_BRICK};
    const int64_t seg0 = a.boff[jo * kLenClasses], seg1 = a.boff[(jo + 1) * kLenClasses];

    // stage the brick's corner records
    for (int p = t; p < kBrickVox; p += kThreads) {
        const int X = b0[0] + p / 81, Y = b0[1] + (p / 9) % 9, Z = b0[2] + p % 9;
        s_id[p] = (X < g.nx && Y < g.ny && Z < g.nz) ? g.index[((int64_t)X * g.ny + Y) * g.nz + Z] : -1;
    }
    __syncthreads();
    for (int k = t; k < kBrickVox * W; k += kThreads) {
        const int p = k / W, w = k - p * W;
        const int id = s_id[p];
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (id >= 0) {
            if constexpr (DT == PLX_F32) {
                const float *rec = static_cast<const float *>(g.data) + (int64_t)id * PLX_REC_SLOTS;
                v = reinterpret_cast<const uint4 *>(rec)[w];
                if (w == 6) v.w = __float_as_uint(rec[PLX_SLOT_SIGMA]);  // slot 27 is padding
            } else {
                v = reinterpret_cast<const uint4 *>(static_cast<const char *>(g.data) +
                                                    (int64_t)id * kRec16Bytes)[w];
            }
        }
        s_rec[k] = v;
    }
    __syncthreads();

    // march the brick's segments, one lane each
    for (int64_t i = seg0 + t; i < seg1; i += kThreads) {
        const int4 sg = a.bseg[i];
        if (!seg_valid(a, sg, a.n_seg)) continue;
        float o[3], d[3];
        load_ray_lane(a, sg.x, o, d);
        RayGeom r;
        const int n = ray_setup(g, o, d, r);
        float y[9];
        sh_basis_all(d, y);
        CornerCache cc;
        cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
        SpanCursor cur{sg.y, 0, 0u};
        double tau = 0.0;
        float C[3] = {0.0f, 0.0f, 0.0f};
        int64_t base = 0, room = 0;
        if (REC) {
            base = a.soff[i];
            room = (int64_t)sg.z - sg.y + 1;
            if (base < 0 || base + room > a.samp_cap) room = 0;
        }
        int j = 0;
        while (true) {
            const int k = span_next_up(g, r, n, sg.z, cur);
            if (k < 0) break;
            const Sample s = sample_at(g, r, k);
            move_staged<DT>(cc, s.cell, b0, s_rec, s_id, y);
            float w[8];
            corner_weights(s.f, w);
            const Q4 v = interpolate(cc, w);
            if (REC && j < room) {
                const int code = (k << 9) | ((s.cell[0] & (PLX_BRICK - 1)) << 6) |
                                 ((s.cell[1] & (PLX_BRICK - 1)) << 3) | (s.cell[2] & (PLX_BRICK - 1));
                SampleRec *rec = a.srec + base + j;
                rec->pos = make_float4(s.f[0], s.f[1], s.f[2], __int_as_float(code));
                rec->val = make_float4(v.s, v.r, v.g, v.b);
            }
            ++j;
            const float sd = fmaxf(v.s, 0.0f) * s.delta;
            const float wk = expf(-(float)tau) * (-expm1f(-sd));
            C[0] += wk * fmaxf(v.r, 0.0f);
            C[1] += wk * fmaxf(v.g, 0.0f);
            C[2] += wk * fmaxf(v.b, 0.0f);
            tau += (double)sd;
        }
        a.tau_seg[sg.w] = tau;
        a.c_seg[sg.w] = make_float4(C[0], C[1], C[2], 0.0f);
        if (REC) a.nocc[i] = (int)min((int64_t)j, room);
    }
}

// ------------------------------------------------------------ sample-parallel forward
//
// The recording forward of the training call, one workgroup per brick with
// segments, in three phases per group of up to kFwdSegs of its segments:
//  1. two or four lanes per segment (one for a large group) walk its
//     samples in runs of kWalkRun and store each occupied one's position
//     record (position in its cell, sample index, cell) in the segment's
//     slots of the sample buffer, in sample order; the waves with no
//     segment meanwhile load the brick's corner ids and first staging;
//  2. every lane takes samples of the group (all lanes busy, whatever the
//     segments' lengths) and interpolates them from the brick's corner
//     records, staged in LDS (FP32 in two halves along x of 5 x 9 x 9
//     corners, 45 KB, so that two workgroups fit on a CU; 16-bit records
//     whole), storing the values in the sample's record;
//  3. the lanes of a segment compose runs of its records, each with the
//     transmittance from the run's start, and chain the runs (a run's colour
//     times the transmittance of the runs before it).
// The values and the composition are those of seg_fwd (project each corner
// on the ray's SH basis, trilinear weights, Eq. (1) with the FP64 optical
// depth); the assignment of work to lanes and the grouping of the
// composition's products differ.

constexpr int kFwdThreads = 512;  // threads of a forward workgroup
constexpr int kFwdSegs = 512;     // segments per group
constexpr int kWalkRun = 8;       // consecutive samples a walking lane tests at once
// Segments per brick (on average over the call) from which the training call
// takes this forward: with fewer, most of a 512-thread workgroup idles in the
// walk and the composition, and the lane-per-segment forward is faster (on
// the 512^3 / 5% grid: 0.35 against 0.72 ms at 65,536 rays, about 9
// segments per brick; even at 262,144 rays, about 36; 2.66 against 1.81 ms
// at 1M rays, 138)
constexpr int64_t kFwdParMinSegs = 40;

template <int DT> struct FwdStage {
    static constexpr int kHalves = DT == PLX_F32 ? 2 : 1;
    static constexpr int kPlanes = PLX_BRICK / kHalves + 1;  // corner planes along x per half
    static constexpr int kWords = StagedRec<DT>::kWords;
    static constexpr int kVox = kPlanes * 81;
    // samples a thread keeps across the halves (FP32: two, within 128 registers)
    static constexpr int kPer = DT == PLX_F32 ? 2 : 4;
    static constexpr int kChunk = kPer * kFwdThreads;
};

// Stages the corner records of planes x = x0 .. x0 + kPlanes - 1 of the
// brick's 9^3 lattice (NULL corners as zeros).
template <int DT>
__device__ __forceinline__ void stage_planes(const GridDev &g, uint4 *s_rec, const int *s_id, int x0) {
    constexpr int W = FwdStage<DT>::kWords;
    for (int k = threadIdx.x; k < FwdStage<DT>::kVox * W; k += kFwdThreads) {
        const int p = k / W, w = k - p * W;
        const int id = s_id[x0 * 81 + p];
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (id >= 0) {
            if constexpr (DT == PLX_F32) {
                const float *rec = static_cast<const float *>(g.data) + (int64_t)id * PLX_REC_SLOTS;
                v = reinterpret_cast<const uint4 *>(rec)[w];
                if (w == 6) v.w = __float_as_uint(rec[PLX_SLOT_SIGMA]);  // slot 27 is padding
            } else {
                v = reinterpret_cast<const uint4 *>(static_cast<const char *>(g.data) +
                                                    (int64_t)id * kRec16Bytes)[w];
            }
        }
        s_rec[k] = v;
    }
}

// The staged words of the corner record with id `id` (NULL: zeros).
template <int DT>
__device__ __forceinline__ void load_corner_words(const GridDev &g, int id, uint4 wv[]) {
    constexpr int W = StagedRec<DT>::kWords;
#pragma unroll
    for (int w = 0; w < W; ++w) wv[w] = make_uint4(0u, 0u, 0u, 0u);
    if (id < 0) return;
    if constexpr (DT == PLX_F32) {
        const float *rec = static_cast<const float *>(g.data) + (int64_t)id * PLX_REC_SLOTS;
#pragma unroll
        for (int w = 0; w < W; ++w) wv[w] = reinterpret_cast<const uint4 *>(rec)[w];
        wv[W - 1].w = __float_as_uint(rec[PLX_SLOT_SIGMA]);  // slot 27 is padding
    } else {
        const uint4 *rec = reinterpret_cast<const uint4 *>(static_cast<const char *>(g.data) +
                                                           (int64_t)id * kRec16Bytes);
#pragma unroll
        for (int w = 0; w < W; ++w) wv[w] = rec[w];
    }
}

// Loads the ids of the brick's 9^3 corners into s_id and the records of the
// first staging (planes 0 .. kPlanes-1) into s_rec; thread `start` of
// `stride` threads takes corners start, start + stride, ...
template <int DT>
__device__ __forceinline__ void stage_ids_first(const GridDev &g, const int b0[3], int *s_id, uint4 *s_rec,
                                                int start, int stride) {
    constexpr int W = StagedRec<DT>::kWords;
    for (int p = start; p < kBrickVox; p += stride) {
        const int X = b0[0] + p / 81, Y = b0[1] + (p / 9) % 9, Z = b0[2] + p % 9;
        const int id = (X < g.nx && Y < g.ny && Z < g.nz) ? g.index[((int64_t)X * g.ny + Y) * g.nz + Z] : -1;
        s_id[p] = id;
        if (p < FwdStage<DT>::kVox) {
            uint4 wv[W];
            load_corner_words<DT>(g, id, wv);
#pragma unroll
            for (int w = 0; w < W; ++w) s_rec[p * W + w] = wv[w];
        }
    }
}

template <int DT>
__global__ __launch_bounds__(kFwdThreads) __attribute__((amdgpu_waves_per_eu(4)))
void seg_fwd_samples_kernel(GridDev g, BinArgs a) {
    using FS = FwdStage<DT>;
    constexpr int W = FS::kWords;
    __shared__ uint4 s_rec[FS::kVox * W];
    __shared__ int s_id[kBrickVox];
    __shared__ float4 s_y4[kFwdSegs * 3];      // SH basis of each segment's ray (9 of 12 floats)
    __shared__ int s_pre[kFwdSegs + 1];        // first sample of each segment in the group's numbering
    __shared__ int64_t s_soff[kFwdSegs];       // its first sample slot
    if (blockIdx.x >= (unsigned)a.n_brick) return;
    const int t = threadIdx.x;
    float *s_y = reinterpret_cast<float *>(s_y4);
    const int64_t jo = a.blist[blockIdx.x];
    const int nty = (g.by + kTile - 1) / kTile, ntz = (g.bz + kTile - 1) / kTile;
    const int64_t tile = jo / (kTile * kTile * kTile);
    const int in = (int)(jo % (kTile * kTile * kTile));
    const int b0[3] = {((int)(tile / ((int64_t)nty * ntz)) * kTile + in / (kTile * kTile)) * PLX_BRICK,
                       ((int)((tile / ntz) % nty) * kTile + (in / kTile) % kTile) * PLX_BRICK,
                       ((int)(tile % ntz) * kTile + in % kTile) * PLX_BRICK};
    const int64_t seg0 = a.boff[jo * kLenClasses], seg1 = a.boff[(jo + 1) * kLenClasses];
    int cur_half = -1;  // half whose corners are in LDS

    for (int64_t c0 = seg0; c0 < seg1; c0 += kFwdSegs) {
        const int ns = (int)min((int64_t)kFwdSegs, seg1 - c0);
        // 1. walk: kL lanes per segment (lane t: segment t / kL, part t % kL),
        // each taking runs of kWalkRun consecutive samples, store the
        // segment's occupied sample positions in order
        const int kL = ns * 4 <= kFwdThreads - 2 * kWave ? 4 : (ns * 2 <= kFwdThreads - 2 * kWave ? 2 : 1);
        const int sx = t / kL, part = t % kL;
        const bool mine = sx < ns;
        const int64_t i = c0 + sx;
        int4 sg = make_int4(0, 0, -1, 0);
        bool live = false;
        RayGeom r = {};
        int occ = 0;
        int64_t base = 0;
        // the waves with no segment of the first group load the corner ids
        // and the first staging meanwhile
        const int st0 = (ns * kL + kWave - 1) / kWave * kWave;
        const bool pre_stage = cur_half < 0 && st0 < kFwdThreads;
        if (pre_stage && t >= st0) stage_ids_first<DT>(g, b0, s_id, s_rec, t - st0, kFwdThreads - st0);
        if (mine) {
            sg = a.bseg[i];
            base = a.soff[i];
            float o[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
            live = seg_valid(a, sg, a.n_seg);
            if (live) {
                load_ray_lane(a, sg.x, o, d);
                const int n = ray_setup(g, o, d, r);
                const int64_t room = (int64_t)sg.z - sg.y + 1;  // the slots the count reserved
                if (base >= 0 && base + room <= a.samp_cap) {
                    // the kL lanes of a segment are adjacent and loop together
                    for (int kr = sg.y; kr <= sg.z; kr += kL * kWalkRun) {
                        const int ks = kr + part * kWalkRun;
                        uint32_t bits = 0u;
                        if (ks <= sg.z) {
                            bits = chunk_bits<kWalkRun>(g, r, n, ks);
                            if (sg.z - ks < kWalkRun - 1) bits &= (2u << (sg.z - ks)) - 1u;
                        }
                        const int c = __popc(bits);
                        int incl = c;  // inclusive prefix over the segment's parts
                        for (int dd = 1; dd < kL; dd <<= 1) {
                            const int y = __shfl_up(incl, dd, kL);
                            if (part >= dd) incl += y;
                        }
                        const int all = __shfl(incl, kL - 1, kL);
                        int at = occ + incl - c;
                        while (bits != 0u) {
                            const int k = ks + __builtin_ctz(bits);
                            bits &= bits - 1u;
                            const Sample sm = sample_at(g, r, k);
                            const int code = (k << 9) | ((sm.cell[0] & (PLX_BRICK - 1)) << 6) |
                                             ((sm.cell[1] & (PLX_BRICK - 1)) << 3) | (sm.cell[2] & (PLX_BRICK - 1));
                            a.srec[base + at].pos = make_float4(sm.f[0], sm.f[1], sm.f[2], __int_as_float(code));
                            ++at;
                        }
                        occ += all;
                    }
                }
            }
            if (part == 0) {
                sh_basis_all(d, s_y + sx * 12);
                s_soff[sx] = base;
            }
        }
        if (cur_half < 0) {
            if (!pre_stage) {
                // no wave was free during the walk: all threads stage
                stage_ids_first<DT>(g, b0, s_id, s_rec, t, kFwdThreads);
            }
            cur_half = 0;
        }
        int64_t tot64;
        const int pre = (int)block_scan_excl<kFwdThreads>(mine && part == 0 ? occ : 0, &tot64);
        const int tot = (int)tot64;
        if (mine && part == 0) s_pre[sx] = pre;
        if (t == 0) s_pre[kFwdSegs] = tot;
        __syncthreads();  // positions stored, s_pre / s_soff / s_y / the staging written

        // 2. values: FS::kPer samples per thread per chunk; the chunk takes the
        // halves starting with the one in LDS
        for (int q0 = 0; q0 < tot; q0 += FS::kChunk) {
            int seg_u[FS::kPer];
            int64_t slot_u[FS::kPer];
            float4 pos_u[FS::kPer];
#pragma unroll
            for (int u = 0; u < FS::kPer; ++u) {
                const int q = q0 + u * kFwdThreads + t;
                seg_u[u] = -1;
                slot_u[u] = 0;
                if (q < tot) {
                    int lo = 0, hi = ns - 1;  // last segment whose first sample is <= q
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= q) lo = mid;
                        else hi = mid - 1;
                    }
                    seg_u[u] = lo;
                    slot_u[u] = s_soff[lo] + (q - s_pre[lo]);
                }
            }
#pragma unroll
            for (int u = 0; u < FS::kPer; ++u)
                if (seg_u[u] >= 0) pos_u[u] = a.srec[slot_u[u]].pos;
            for (int hh = 0; hh < FS::kHalves; ++hh) {
                const int h = (cur_half + hh) % FS::kHalves;
                if (h != cur_half) {
                    __syncthreads();  // the other half's reads are done
                    stage_planes<DT>(g, s_rec, s_id, h * (FS::kPlanes - 1));
                    __syncthreads();
                    cur_half = h;
                }
#pragma unroll
                for (int u = 0; u < FS::kPer; ++u) {
                    if (seg_u[u] < 0) continue;
                    const int code = __float_as_int(pos_u[u].w);
                    const int cx = (code >> 6) & (PLX_BRICK - 1), cy = (code >> 3) & (PLX_BRICK - 1),
                              cz = code & (PLX_BRICK - 1);
                    const int lx = cx - h * (FS::kPlanes - 1);
                    if (lx < 0 || lx >= FS::kPlanes - 1) continue;  // the sample's cell is in the other half
                    float y[9];
#pragma unroll
                    for (int l = 0; l < 9; ++l) y[l] = s_y[seg_u[u] * 12 + l];
                    const float f[3] = {pos_u[u].x, pos_u[u].y, pos_u[u].z};
                    float w[8];
                    corner_weights(f, w);
                    Q4 v = q4_zero();
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int p = (lx + ((c >> 2) & 1)) * 81 + (cy + ((c >> 1) & 1)) * 9 + (cz + (c & 1));
                        const Q4 qc = project_staged<DT>(s_rec + p * W, y);
                        v.s += w[c] * qc.s;
                        v.r += w[c] * qc.r;
                        v.g += w[c] * qc.g;
                        v.b += w[c] * qc.b;
                    }
                    a.srec[slot_u[u]].val = make_float4(v.s, v.r, v.g, v.b);
                }
            }
        }
        __syncthreads();  // every value stored before the segments compose

        // 3. composition: the kL lanes of a segment each compose a run of its
        // samples (transmittance from the run's start, record loads kCompU at
        // a time), then the runs are chained: run q's colour is scaled by the
        // transmittance of the runs before it (a segment without slots, which
        // the emit walk reports in the status word, contributes nothing)
        if (mine && live) {
            constexpr int kCompU = 4;
            const int per = (occ + kL - 1) / kL;
            const int j_lo = min(occ, part * per), j_hi = min(occ, j_lo + per);
            double tau = 0.0;
            float C[3] = {0.0f, 0.0f, 0.0f};
            for (int j0 = j_lo; j0 < j_hi; j0 += kCompU) {
                SampleRec rb[kCompU];
#pragma unroll
                for (int u = 0; u < kCompU; ++u)
                    if (j0 + u < j_hi) rb[u] = a.srec[base + j0 + u];
#pragma unroll
                for (int u = 0; u < kCompU; ++u) {
                    if (j0 + u >= j_hi) break;
                    const int k = (int)((unsigned)__float_as_int(rb[u].pos.w) >> 9);
                    const float delta = sample_at(g, r, k).delta;
                    const float sd = fmaxf(rb[u].val.x, 0.0f) * delta;
                    const float wk = expf(-(float)tau) * (-expm1f(-sd));
                    C[0] += wk * fmaxf(rb[u].val.y, 0.0f);
                    C[1] += wk * fmaxf(rb[u].val.z, 0.0f);
                    C[2] += wk * fmaxf(rb[u].val.w, 0.0f);
                    tau += (double)sd;
                }
            }
            if (kL > 1) {
                double incl = tau;  // optical depth up to the end of this run
                for (int dd = 1; dd < kL; dd <<= 1) {
                    const double y = __shfl_up(incl, dd, kL);
                    if (part >= dd) incl += y;
                }
                const float T0 = expf(-(float)(incl - tau));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    C[c] *= T0;
                    for (int dd = 1; dd < kL; dd <<= 1) C[c] += __shfl_xor(C[c], dd, kL);
                }
                tau = __shfl(incl, kL - 1, kL);
            }
            if (part == 0) {
                a.tau_seg[sg.w] = tau;
                a.c_seg[sg.w] = make_float4(C[0], C[1], C[2], 0.0f);
                a.nocc[i] = occ;
            }
        }
        __syncthreads();  // s_y / s_pre / s_soff are rewritten by the next group
    }
}

// Segments of a ray are walked kSegU at a time: the loads of a group are
// issued together (positions past the last segment are clamped to it and
// their values unused), then the group is composed in order.
constexpr int kSegU = 4;

// Per ray: composes its segments into the colour (and optical depth).  FWD
// writes them out; TRAIN also forms the loss and dL/dC = 2 loss_scale (C -
// target), BWD takes dL/dC as given; both then record, for every segment,
// the optical depth before it and g . R after it.
template <int MODE>
__global__ __launch_bounds__(kThreads) void seg_combine_kernel(BinArgs a) {
    __shared__ double blk_loss[kWavesPerBlock];
    const int64_t ray = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double l2 = 0.0, lb = 0.0;
    if constexpr (MODE == MODE_MAXW) {
        if (ray < a.n_rays) {
            const int64_t s0 = a.seg_off[ray], s1 = min(a.seg_off[ray + 1], a.seg_cap);
            double tau = 0.0;
            for (int64_t s = s0; s < s1; s += kSegU) {
                double ts[kSegU];
#pragma unroll
                for (int u = 0; u < kSegU; ++u) ts[u] = a.tau_seg[min(s + u, s1 - 1)];
#pragma unroll
                for (int u = 0; u < kSegU; ++u) {
                    if (s + u < s1) {
                        a.tau_in[s + u] = tau;
                        tau += ts[u];
                    }
                }
            }
        }
        return;
    }
    if (ray < a.n_rays) {
        const int64_t s0 = a.seg_off[ray], s1 = min(a.seg_off[ray + 1], a.seg_cap);
        double tau = 0.0;
        float C[3] = {0.0f, 0.0f, 0.0f};
        for (int64_t s = s0; s < s1; s += kSegU) {
            double ts[kSegU];
            float4 cs[kSegU];
#pragma unroll
            for (int u = 0; u < kSegU; ++u) {
                const int64_t sc = min(s + u, s1 - 1);
                ts[u] = a.tau_seg[sc];
                cs[u] = a.c_seg[sc];
            }
#pragma unroll
            for (int u = 0; u < kSegU; ++u) {
                if (s + u < s1) {
                    if (MODE != MODE_FWD) a.tau_in[s + u] = tau;
                    const float T = expf(-(float)tau);
                    C[0] += T * cs[u].x;
                    C[1] += T * cs[u].y;
                    C[2] += T * cs[u].z;
                    tau += ts[u];
                }
            }
        }
        const float T_final = expf(-(float)tau);
        float gr[3], R[3], bgc[3];
        ray_background(a.bg_rgb, a.bg, ray, bgc);
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) {
            const float Cc = C[c3] + T_final * bgc[c3];
            if (MODE != MODE_BWD && a.rgb_out) a.rgb_out[3 * ray + c3] = Cc;
            if (MODE == MODE_TRAIN) {
                const float diff = Cc - a.target[3 * ray + c3];
                gr[c3] = 2.0f * a.loss_scale * diff;
                l2 += (double)(diff * diff);
            } else if (MODE == MODE_BWD) {
                gr[c3] = a.grad_rgb[3 * ray + c3];
            }
            R[c3] = T_final * bgc[c3];
        }
        if (MODE == MODE_FWD) {
            if (a.tau_out) a.tau_out[ray] = (float)tau;
        } else {
            const float gw = a.pri.lambda_b != 0.0f ? beta_factor(a.pri, tau, &lb) : 0.0f;
            a.g_ray[ray] = make_float4(gr[0], gr[1], gr[2], gw);
            if (a.grad_bg) {
#pragma unroll
                for (int c3 = 0; c3 < 3; ++c3) a.grad_bg[3 * ray + c3] = T_final * gr[c3];
            }
            for (int64_t s = s1 - 1; s >= s0; s -= kSegU) {
                double ti[kSegU];
                float4 cs[kSegU];
#pragma unroll
                for (int u = 0; u < kSegU; ++u) {
                    const int64_t sc = max(s - u, s0);
                    ti[u] = a.tau_in[sc];
                    cs[u] = a.c_seg[sc];
                }
#pragma unroll
                for (int u = 0; u < kSegU; ++u) {
                    if (s - u >= s0) {
                        a.gr_after[s - u] = gr[0] * R[0] + gr[1] * R[1] + gr[2] * R[2];
                        const float T = expf(-(float)ti[u]);
                        R[0] += T * cs[u].x;
                        R[1] += T * cs[u].y;
                        R[2] += T * cs[u].z;
                    }
                }
            }
        }
    }
    if (MODE != MODE_FWD) add_prior_loss(a.pri, 0.0f, lb);
    if (MODE == MODE_TRAIN) {
        double wl = (double)a.loss_scale * l2;
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) wl += __shfl_xor(wl, m);
        if ((threadIdx.x & (kWave - 1)) == 0) blk_loss[threadIdx.x / kWave] = wl;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kWavesPerBlock; ++w) t += blk_loss[w];
            if (t != 0.0) unsafeAtomicAdd(a.loss_sum, t);
        }
    }
}

// Backward replay of one segment, from its last occupied sample to its first.
template <int DT, bool CAUCHY>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
void seg_bwd_kernel(GridDev g, BinArgs a) {
    __shared__ int q_count[kWavesPerBlock];
    __shared__ int q_id[kWavesPerBlock * kQCap];
    __shared__ uint8_t q_src[kWavesPerBlock * kQCap];
    __shared__ float4 q_v[kWavesPerBlock * kQCap];
    __shared__ float q_y[kWavesPerBlock * kWave * 9];

    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int wid = threadIdx.x / kWave;
    const int L = lane_id();
    if (L == 0) q_count[wid] = 0;
    __syncthreads();
    Queue qu;
    qu.count = q_count + wid;
    qu.id = q_id + wid * kQCap;
    qu.src = q_src + wid * kQCap;
    qu.v = q_v + wid * kQCap;
    qu.y = q_y + wid * kWave * 9;

    const int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    const int64_t n_seg = seg_count_of(a);
    int4 sg = make_int4(0, 0, -1, 0);
    if (i < n_seg) sg = a.bseg[i];
    const bool live = i < n_seg && seg_valid(a, sg, n_seg);
    float o[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
    if (live) load_ray_lane(a, sg.x, o, d);
    RayGeom r;
    const int n = live ? ray_setup(g, o, d, r) : 0;
    float *y = qu.y + L * 9;
    sh_basis_all(d, y);

    CornerCache cc;
    cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
    Q4 acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = q4_zero();

    float gr[3] = {0.f, 0.f, 0.f};
    double tau_after = 0.0;
    float gR = 0.0f, ls = 0.0f;
    if (live) {
        const float4 gg = a.g_ray[sg.x];
        gr[0] = gg.x;
        gr[1] = gg.y;
        gr[2] = gg.z;
        tau_after = a.tau_in[sg.w] + a.tau_seg[sg.w];
        gR = a.gr_after[sg.w] - gg.w;  // the beta factor joins the running sum
    }
    float T_after = expf(-(float)tau_after);
    SpanCursor cur{sg.z, 0, 0u};
    bool active = live && n > 0;
    while (__any(active)) {
        if (active) {
            const int k = span_next_down(g, r, n, sg.y, cur);
            if (k < 0) {
                if (cc.cell[0] >= 0) push_corners(qu, cc, acc, 0xffu);
                active = false;
            } else {
                const Sample s = sample_at(g, r, k);
                move_to<DT, true>(g, cc, s.cell, acc, qu, y);
                float w[8];
                corner_weights(s.f, w);
                const Q4 v = interpolate(cc, w);
                const float sd = fmaxf(v.s, 0.0f) * s.delta;
                const double tau_before = fmax(tau_after - (double)sd, 0.0);
                const float T_before = expf(-(float)tau_before);
                const float wk = T_before * (-expm1f(-sd));
                const float gc = gr[0] * fmaxf(v.r, 0.0f) + gr[1] * fmaxf(v.g, 0.0f) +
                                 gr[2] * fmaxf(v.b, 0.0f);
                const float cs = CAUCHY ? cauchy_grad(a.pri, v.s, &ls) : 0.0f;
                const float dsig = v.s > 0.0f ? s.delta * (T_after * gc - gR) + cs : 0.0f;
                const float g_r = v.r > 0.0f ? wk * gr[0] : 0.0f;
                const float g_g = v.g > 0.0f ? wk * gr[1] : 0.0f;
                const float g_b = v.b > 0.0f ? wk * gr[2] : 0.0f;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    acc[c].s += w[c] * dsig;
                    acc[c].r += w[c] * g_r;
                    acc[c].g += w[c] * g_g;
                    acc[c].b += w[c] * g_b;
                }
                gR += wk * gc;
                tau_after = tau_before;
                T_after = T_before;
            }
        }
        drain(qu, a.grad, a.touched);
    }
    if (CAUCHY) add_prior_loss(a.pri, ls, 0.0);
}

// ------------------------------------------------------------ recorded backward
//
// The scatter of seg_bwd sends about nine partial gradients to every voxel a
// batch reaches (one per segment that has it as a corner), each a 128-B line
// of FP32 atomics, and global atomics are the slowest path on the chip (about
// 20G 64-byte requests per second, whatever the lanes' pattern); its replay
// also repeats the forward's corner gathers.  The recorded backward instead:
//  1. seg_fwd (REC) stores, per occupied sample, its position in the cell,
//     sample index, cell and interpolated values (32 B) in the segment's
//     slots of the sample buffer;
//  2. seg_combine forms the per-ray and per-segment quantities as before;
//  3. seg_scatter (one workgroup per brick with segments) loads the brick's
//     samples into LDS, runs each segment's reverse recurrence over them
//     (one lane per segment: transmittance from the FP64 optical depth after
//     the segment, the radiance collected after it, the sample's gradients
//     with respect to its density and projected colour), sorts the samples
//     by cell, and then each lane owns one of the brick's 9^3 corner voxels
//     and sums the contributions of the samples of the (up to) 8 cells around
//     it, so every voxel gets one 128-B line of atomics per brick instead of
//     one per segment, and no corner record is read a second time.
// The terms are those of seg_bwd (Sec. 3.3, Eq. (1) and the chain rule
// through the trilinear weights and the SH basis); only the order of the
// additions differs.

constexpr int kScatterThreads = 512;       // threads of a scatter workgroup
constexpr int kScatterSegs = 256;          // segments per pass
constexpr int kVoxRounds = (kBrickVox + kScatterThreads - 1) / kScatterThreads;
constexpr int kScatterCap = 1536;          // samples in LDS per pass
constexpr int kScatterPer = kScatterCap / kScatterThreads;
constexpr int kStageRows = 8;              // rows a wave stages per flush round
constexpr int kStageStride = 29;           // 28 values and the voxel id per staged row

// A sample in the scatter's LDS.  Before the sort: v = the interpolated
// values, then (after the recurrence) the gradients; code = sample index and
// cell.  After the sort: f, the gradients in v, and seg = the pass-local
// number of its segment.
struct LdsSample {
    float f[3];
    float v[4];
    int seg;
};
static_assert(sizeof(LdsSample) == 32, "two 16-byte words per sample");

// Sends the 28 gradient values of every lane's voxel (id < 0: none) to the
// FP32 records, kStageRows rows at a time through the wave's staging rows:
// lanes 0..31 then take one row and lanes 32..63 the next, lane s of a half
// the record slot s (0..26 SH, 28 density, 29 the touched byte), so every
// instruction covers two 128-B gradient lines.  Called by the whole wave.
__device__ __forceinline__ void flush_voxel_rows(float *stage, const float acc[28], int id, float *grad,
                                                 uint8_t *touched) {
    const int L = lane_id();
    const int s = L & 31;
    const int half = L >> 5;
    const int col = s < PLX_NSH ? s : PLX_NSH;  // staged column of the lane's slot
#pragma unroll
    for (int h = 0; h < kWave / kStageRows; ++h) {
        const bool mine = L / kStageRows == h;
        if (__ballot(id >= 0 && mine) == 0) continue;
        if (mine) {
            float *row = stage + (L % kStageRows) * kStageStride;
#pragma unroll
            for (int v = 0; v < 28; ++v) row[v] = acc[v];
            row[28] = __int_as_float(id);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < kStageRows / 2; ++u) {
            const float *row = stage + (2 * u + half) * kStageStride;
            const int rid = __float_as_int(row[28]);
            const float val = row[col];
            if (rid >= 0) {
                if ((s < PLX_NSH || s == PLX_SLOT_SIGMA) && val != 0.0f)
                    unsafeAtomicAdd(grad + (int64_t)rid * PLX_REC_SLOTS + s, val);
                if (s == PLX_SLOT_SIGMA + 1) touched[rid] = 1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Reverse recurrence of one segment (the state a lane carries along it).
struct SegState {
    double tau_after;  // optical depth after the current sample
    float T_after;
    float gR;          // g . (radiance collected after the current sample)
    float gr[3];       // dL/dC of the ray
    float ls;          // Cauchy prior loss of the lane
};

template <bool CAUCHY>
__global__ __launch_bounds__(kScatterThreads) __attribute__((amdgpu_waves_per_eu(4)))
void seg_scatter_kernel(GridDev g, BinArgs a) {
    __shared__ int64_t s_soff[kScatterSegs];   // sample slot of each segment of the group
    __shared__ int s_pre[kScatterSegs + 1];    // its first sample in the group's numbering
    __shared__ float4 s_y4[kScatterSegs * 3];  // SH basis of its ray (9 of 12 floats)
    __shared__ int s_cnt[kBrickCells];         // samples per cell
    __shared__ int s_coff[kBrickCells + 1];    // first sorted position of each cell
    __shared__ __align__(16) LdsSample s_rec[kScatterCap];   // the pass's samples
    __shared__ float s_stage[kScatterThreads / kWave * kStageRows * kStageStride];

    if (blockIdx.x >= (unsigned)a.n_brick) return;
    const int t = threadIdx.x;
    float *s_y = reinterpret_cast<float *>(s_y4);
    float *stage = s_stage + (t / kWave) * kStageRows * kStageStride;
    // brick coordinates from its position in the binning order
    const int64_t jo = a.blist[blockIdx.x];
    const int nty = (g.by + kTile - 1) / kTile, ntz = (g.bz + kTile - 1) / kTile;
    const int64_t tile = jo / (kTile * kTile * kTile);
    const int in = (int)(jo % (kTile * kTile * kTile));
    const int bxyz[3] = {(int)(tile / ((int64_t)nty * ntz)) * kTile + in / (kTile * kTile),
                         (int)((tile / ntz) % nty) * kTile + (in / kTile) % kTile,
                         (int)(tile % ntz) * kTile + in % kTile};
    const int64_t seg0 = a.boff[jo * kLenClasses], seg1 = a.boff[(jo + 1) * kLenClasses];

    // the lane's corner voxels (position p = x*81 + y*9 + z of the 9^3 lattice)
    int vid[kVoxRounds];
#pragma unroll
    for (int rr = 0; rr < kVoxRounds; ++rr) {
        const int p = t + rr * kScatterThreads;
        vid[rr] = -1;
        if (p < kBrickVox) {
            const int X = bxyz[0] * PLX_BRICK + p / 81, Y = bxyz[1] * PLX_BRICK + (p / 9) % 9,
                      Z = bxyz[2] * PLX_BRICK + p % 9;
            if (X < g.nx && Y < g.ny && Z < g.nz) vid[rr] = g.index[((int64_t)X * g.ny + Y) * g.nz + Z];
        }
    }
    float ls = 0.0f;

    for (int64_t c0 = seg0; c0 < seg1; c0 += kScatterSegs) {
        // a group of up to kScatterSegs segments; lane t < ns walks segment t
        const int ns = (int)min((int64_t)kScatterSegs, seg1 - c0);
        int occ = 0;
        int4 sg = make_int4(0, 0, -1, 0);
        SegState st = {};
        if (t < ns) {
            const int64_t i = c0 + t;
            sg = a.bseg[i];
            float d[3] = {0.f, 0.f, 1.f};
            if (seg_valid(a, sg, a.n_seg)) {
                occ = a.nocc[i];
                d[0] = a.rays_d[3 * (int64_t)sg.x];
                d[1] = a.rays_d[3 * (int64_t)sg.x + 1];
                d[2] = a.rays_d[3 * (int64_t)sg.x + 2];
                const float4 gg = a.g_ray[sg.x];
                st.gr[0] = gg.x;
                st.gr[1] = gg.y;
                st.gr[2] = gg.z;
                st.tau_after = a.tau_in[sg.w] + a.tau_seg[sg.w];
                st.gR = a.gr_after[sg.w] - gg.w;  // the beta factor joins the running sum
                st.T_after = expf(-(float)st.tau_after);
            }
            s_soff[t] = a.soff[i];
            sh_basis_all(d, s_y + t * 12);
        }
        int64_t tot64;
        const int pre = (int)block_scan_excl<kScatterThreads>(occ, &tot64);
        const int tot = (int)tot64;
        if (t < kScatterSegs) s_pre[t] = pre;  // segments past ns hold the total
        if (t == 0) s_pre[kScatterSegs] = tot;
        __syncthreads();

        // passes over the group's samples from the last one back, so that a
        // segment longer than a pass meets its samples in reverse order
        for (int q0 = ((tot - 1) / kScatterCap) * kScatterCap; tot > 0 && q0 >= 0; q0 -= kScatterCap) {
            const int nq = min(kScatterCap, tot - q0);
            for (int c = t; c < kBrickCells; c += kScatterThreads) s_cnt[c] = 0;
            // load the pass's samples (slots first, then all loads), count them
            // per cell and leave them unsorted in LDS for the recurrence
            int seg_u[kScatterPer];
            int64_t slot_u[kScatterPer];
#pragma unroll
            for (int u = 0; u < kScatterPer; ++u) {
                const int q = u * kScatterThreads + t;
                seg_u[u] = -1;
                slot_u[u] = 0;
                if (q < nq) {
                    const int qq = q0 + q;
                    int lo = 0, hi = ns - 1;  // last segment whose first sample is <= qq
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pre[mid] <= qq) lo = mid;
                        else hi = mid - 1;
                    }
                    seg_u[u] = lo;
                    slot_u[u] = s_soff[lo] + (qq - s_pre[lo]);
                }
            }
            SampleRec rec_u[kScatterPer];
#pragma unroll
            for (int u = 0; u < kScatterPer; ++u)
                if (seg_u[u] >= 0) rec_u[u] = a.srec[slot_u[u]];
            __syncthreads();  // s_cnt cleared; the previous pass's LDS reads done
            int cell_u[kScatterPer], rank_u[kScatterPer];
#pragma unroll
            for (int u = 0; u < kScatterPer; ++u) {
                if (seg_u[u] >= 0) {
                    const int code = __float_as_int(rec_u[u].pos.w);
                    cell_u[u] = code & (kBrickCells - 1);
                    rank_u[u] = atomicAdd(&s_cnt[cell_u[u]], 1);
                    LdsSample &ls_q = s_rec[u * kScatterThreads + t];
                    ls_q.f[0] = rec_u[u].pos.x;
                    ls_q.f[1] = rec_u[u].pos.y;
                    ls_q.f[2] = rec_u[u].pos.z;
                    ls_q.v[0] = rec_u[u].val.x;
                    ls_q.v[1] = rec_u[u].val.y;
                    ls_q.v[2] = rec_u[u].val.z;
                    ls_q.v[3] = rec_u[u].val.w;
                    ls_q.seg = code;
                }
            }
            __syncthreads();
            {
                static_assert(kScatterThreads == kBrickCells, "one cell per thread");
                int64_t all;
                s_coff[t] = (int)block_scan_excl<kScatterThreads>(s_cnt[t], &all);
                if (t == 0) s_coff[kBrickCells] = (int)all;
            }
            // the reverse recurrence of each segment over its samples of the pass
            if (t < ns && occ > 0) {
                const int e_lo = max(s_pre[t], q0) - q0, e_hi = min(s_pre[t] + occ, q0 + nq) - q0;
                if (e_lo < e_hi) {
                    float o[3], d[3];
                    load_ray_lane(a, sg.x, o, d);
                    RayGeom r;
                    const int n = ray_setup(g, o, d, r);
                    (void)n;
                    for (int e = e_hi - 1; e >= e_lo; --e) {
                        LdsSample &sm = s_rec[e];
                        const int k = (unsigned)sm.seg >> 9;
                        const float delta = sample_at(g, r, k).delta;
                        const Q4 v = {sm.v[0], sm.v[1], sm.v[2], sm.v[3]};
                        const float sd = fmaxf(v.s, 0.0f) * delta;
                        const double tau_before = fmax(st.tau_after - (double)sd, 0.0);
                        const float T_before = expf(-(float)tau_before);
                        const float wk = T_before * (-expm1f(-sd));
                        const float gc = st.gr[0] * fmaxf(v.r, 0.0f) + st.gr[1] * fmaxf(v.g, 0.0f) +
                                         st.gr[2] * fmaxf(v.b, 0.0f);
                        const float cs = CAUCHY ? cauchy_grad(a.pri, v.s, &ls) : 0.0f;
                        sm.v[0] = v.s > 0.0f ? delta * (st.T_after * gc - st.gR) + cs : 0.0f;
                        sm.v[1] = v.r > 0.0f ? wk * st.gr[0] : 0.0f;
                        sm.v[2] = v.g > 0.0f ? wk * st.gr[1] : 0.0f;
                        sm.v[3] = v.b > 0.0f ? wk * st.gr[2] : 0.0f;
                        st.gR += wk * gc;
                        st.tau_after = tau_before;
                        st.T_after = T_before;
                    }
                }
            }
            __syncthreads();
            // sort by cell: each thread takes its samples (now with their
            // gradients) back, then puts every one in its cell's range
            LdsSample mine[kScatterPer];
#pragma unroll
            for (int u = 0; u < kScatterPer; ++u)
                if (seg_u[u] >= 0) mine[u] = s_rec[u * kScatterThreads + t];
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kScatterPer; ++u) {
                if (seg_u[u] >= 0) {
                    mine[u].seg = seg_u[u];
                    s_rec[s_coff[cell_u[u]] + rank_u[u]] = mine[u];
                }
            }
            __syncthreads();

            // each lane sums its voxels' contributions and flushes them
#pragma unroll 1
            for (int rr = 0; rr < kVoxRounds; ++rr) {
                const int p = t + rr * kScatterThreads;
                float acc[28];
#pragma unroll
                for (int v = 0; v < 28; ++v) acc[v] = 0.0f;
                // the sample ranges of the voxel's (up to) 8 cells, the
                // non-empty ones first in corner order (start | count << 11 |
                // corner << 22), walked as one list: a wave then runs as long
                // as its busiest lane's total, not the sum over the corners of
                // each corner's busiest lane
                unsigned qr[8];
                int nne = 0;
                {
                    const int px = p / 81, py = (p / 9) % 9, pz = p % 9;
#pragma unroll
                    for (int j = 0; j < 8; ++j) qr[j] = 0u;
#pragma unroll
                    for (int o = 0; o < 8; ++o) {
                        // the voxel is corner o (x: bit 2) of the cell p - o
                        const int cx = px - ((o >> 2) & 1), cy = py - ((o >> 1) & 1), cz = pz - (o & 1);
                        unsigned ent = 0u;
                        if (vid[rr] >= 0 && cx >= 0 && cy >= 0 && cz >= 0 && cx < PLX_BRICK && cy < PLX_BRICK &&
                            cz < PLX_BRICK) {
                            const int cell = (cx << 6) | (cy << 3) | cz;
                            const int c0 = s_coff[cell], n = s_coff[cell + 1] - c0;
                            if (n > 0) ent = (unsigned)c0 | ((unsigned)n << 11) | ((unsigned)o << 22);
                        }
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            if (ent != 0u && j == nne) qr[j] = ent;
                        nne += ent != 0u ? 1 : 0;
                    }
                }
                const bool any = nne > 0;
                int e = (int)(qr[0] & 0x7ffu), cnt = (int)((qr[0] >> 11) & 0x7ffu), oc = (int)(qr[0] >> 22);
#pragma unroll
                for (int j = 0; j < 7; ++j) qr[j] = qr[j + 1];
                qr[7] = 0u;
#pragma unroll 1
                for (;;) {
                    // the wave leaves together; a lane that is done adds nothing
                    const bool live = cnt > 0;
                    if (__ballot(live) == 0) break;
                    // the whole sample in two 16-byte reads, f0 f1 f2 v0 | v1 v2 v3 seg
                    // (a done lane reads sorted sample 0, a valid one)
                    const float4 *sp = reinterpret_cast<const float4 *>(s_rec + (live ? e : 0));
                    const float4 sa = sp[0], sb = sp[1];
                    const float wx = (oc & 4) ? sa.x : 1.0f - sa.x;
                    const float wy = (oc & 2) ? sa.y : 1.0f - sa.y;
                    const float wz = (oc & 1) ? sa.z : 1.0f - sa.z;
                    const float w = wx * wy * wz;
                    const int sy = __float_as_int(sb.w) * 3;
                    const float4 y0 = s_y4[sy], y1 = s_y4[sy + 1], y2 = s_y4[sy + 2];
                    const float yy[9] = {y0.x, y0.y, y0.z, y0.w, y1.x, y1.y, y1.z, y1.w, y2.x};
                    const float a_r = live ? w * sb.x : 0.0f, a_g = live ? w * sb.y : 0.0f,
                                a_b = live ? w * sb.z : 0.0f;
#pragma unroll
                    for (int l = 0; l < 9; ++l) {
                        acc[l] += a_r * yy[l];
                        acc[9 + l] += a_g * yy[l];
                        acc[18 + l] += a_b * yy[l];
                    }
                    const float s27 = acc[27] + w * sa.w;
                    acc[27] = live ? s27 : acc[27];
                    ++e;
                    cnt -= live ? 1 : 0;
                    if (live && cnt == 0) {
                        // next range (an empty entry leaves the lane done)
                        e = (int)(qr[0] & 0x7ffu);
                        cnt = (int)((qr[0] >> 11) & 0x7ffu);
                        oc = (int)(qr[0] >> 22);
#pragma unroll
                        for (int j = 0; j < 7; ++j) qr[j] = qr[j + 1];
                        qr[7] = 0u;
                    }
                }
                flush_voxel_rows(stage, acc, any ? vid[rr] : -1, a.grad, a.touched);
            }
            __syncthreads();
        }
    }
    if (CAUCHY) add_prior_loss(a.pri, ls, 0.0);
}

// ------------------------------------------------------------ maximum sample weight

// Density-only corner cache of the weight pass.  Slot p holds the corner
// whose lattice coordinates have the parities of p's bits (x: bit 2, y: bit 1,
// z: bit 0), so a corner keeps its slot for as long as it stays a corner of
// the current cell and a move never exchanges registers: the slots whose
// corner left are flushed and reloaded.
struct SigmaCache {
    int cell[3];
    int ids[8];
    float s[8];
    float wm[8];  // largest sample weight the corner has seen while cached
};

// Cell offset (corner number, x: bit 2) of the corner in slot p of `cell`.
__device__ __forceinline__ int slot_corner(int p, const int cell[3]) {
    return p ^ (((cell[0] & 1) << 2) | ((cell[1] & 1) << 1) | (cell[2] & 1));
}

// Raises wmax of the cached corners in `mask` (non-negative floats order as
// their bit patterns, so an unsigned maximum is the float maximum).  wmax only
// grows, so a value already at least the candidate makes the atomic
// unnecessary; after the first rays through a brick most candidates are.
__device__ __forceinline__ void flush_max(const SigmaCache &sc, unsigned mask, float *wmax) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        if (((mask >> p) & 1u) && sc.ids[p] >= 0 && sc.wm[p] > 0.0f) {
            unsigned *q = reinterpret_cast<unsigned *>(wmax) + sc.ids[p];
            const unsigned cand = __float_as_uint(sc.wm[p]);
            if (__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < cand) atomicMax(q, cand);
        }
    }
}

// Makes `cell` the cached cell; leaving corners are flushed when MAXW.
template <int DT, bool MAXW>
__device__ __forceinline__ void sigma_move_to(const GridDev &g, SigmaCache &sc, const int cell[3],
                                              float *wmax) {
    if (cell[0] == sc.cell[0] && cell[1] == sc.cell[1] && cell[2] == sc.cell[2]) return;
    const bool had = sc.cell[0] >= 0;
    unsigned stay = 0;
    if (had) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int c = slot_corner(p, cell);
            const unsigned ox = (unsigned)(cell[0] + ((c >> 2) & 1) - sc.cell[0]);
            const unsigned oy = (unsigned)(cell[1] + ((c >> 1) & 1) - sc.cell[1]);
            const unsigned oz = (unsigned)(cell[2] + (c & 1) - sc.cell[2]);
            if (ox <= 1u && oy <= 1u && oz <= 1u) stay |= 1u << p;
        }
        if (MAXW) flush_max(sc, ~stay & 0xffu, wmax);
    }
    sc.cell[0] = cell[0];
    sc.cell[1] = cell[1];
    sc.cell[2] = cell[2];
    const int64_t lin = cell_id(g, sc.cell);
    int nid[8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
        nid[p] = ((stay >> p) & 1u) ? sc.ids[p] : g.index[lin + corner_offset(g, slot_corner(p, cell))];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        if (!((stay >> p) & 1u)) {
            sc.ids[p] = nid[p];
            sc.s[p] = nid[p] >= 0 ? rec_sigma<DT>(g.data, nid[p]) : 0.0f;
            sc.wm[p] = 0.0f;
        }
    }
}

// The weight pass runs in brick order in two phases over the same segments.
// Phase 0 gives each segment's optical depth (density only; no colour is
// needed), the combine step turns those into the depth before each segment,
// and phase 1 replays the segment from there: sample k's weight is
// T_k (1 - exp(-sigma_k delta_k)) with T_k from the ray's running optical
// depth, exactly as the forward pass composites, and every non-NULL corner of
// the sample's cell keeps the largest weight it sees; a corner's maximum goes
// to wmax (one atomic maximum) when it leaves the cache.
template <int DT, int PHASE>
__global__ __launch_bounds__(kThreads) void seg_weight_kernel(GridDev g, BinArgs a) {
    const int blk = xcd_logical_block(blockIdx.x, a.nb8);
    if (blk >= a.n_blocks) return;
    const int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    const int64_t n_seg = seg_count_of(a);
    if (i >= n_seg) return;
    const int4 sg = a.bseg[i];
    if (!seg_valid(a, sg, n_seg)) return;
    float o[3], d[3];
    load_ray_lane(a, sg.x, o, d);
    RayGeom r;
    const int n = ray_setup(g, o, d, r);
    SigmaCache sc;
    sc.cell[0] = sc.cell[1] = sc.cell[2] = -1;
    SpanCursor cur{sg.y, 0, 0u};
    double tau = PHASE == 0 ? 0.0 : a.tau_in[sg.w];
    while (true) {
        const int k = span_next_up(g, r, n, sg.z, cur);
        if (k < 0) break;
        const Sample smp = sample_at(g, r, k);
        sigma_move_to<DT, PHASE == 1>(g, sc, smp.cell, a.wmax);
        // trilinear weights in slot order
        float sp = 0.0f;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int c = slot_corner(p, smp.cell);
            const float ax = (c >> 2) & 1 ? smp.f[0] : 1.0f - smp.f[0];
            const float ay = (c >> 1) & 1 ? smp.f[1] : 1.0f - smp.f[1];
            const float az = c & 1 ? smp.f[2] : 1.0f - smp.f[2];
            sp += ax * ay * az * sc.s[p];
        }
        const float sd = fmaxf(sp, 0.0f) * smp.delta;
        if (PHASE == 1) {
            const float wk = expf(-(float)tau) * (-expm1f(-sd));
#pragma unroll
            for (int p = 0; p < 8; ++p) sc.wm[p] = fmaxf(sc.wm[p], wk);
        }
        tau += (double)sd;
    }
    if (PHASE == 0) a.tau_seg[sg.w] = tau;
    else if (sc.cell[0] >= 0) flush_max(sc, 0xffu, a.wmax);
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

constexpr int kTileW = 16, kTileH = 16;  // pixels per tile = rays per block

// Scene table (device, written by plx_scene_table_set): a 256-byte header,
// then one GridDev per scene.
constexpr unsigned kSceneMagic = 0x504c5853u;
struct SceneTableHeader {
    unsigned magic;
    int n_scenes;
    int sh_dtype;
};
constexpr int64_t kSceneTableHead = 256;

// Views reach the device as kernel arguments (no copy engine, no setup
// launch, no host buffer that must outlive the call): one launch renders up
// to kViewsPerLaunch views, and a longer list is split into several.
constexpr int kViewsPerLaunch = 24;

// The caller's tile queue (PLX_VIEWS_QUEUE_BYTES, zero before first use):
// the next tile, the blocks that have left, and a sticky status word.  The
// last block of a launch to leave resets the first two, so every launch
// finds the queue at zero without a memset.
struct ViewsQueue {
    unsigned long long next;
    unsigned done;
    unsigned status;
};

struct ViewsArgs {
    const SceneTableHeader *table;
    const GridDev *scenes;
    plx_view v[kViewsPerLaunch];
    int64_t tile_start[kViewsPerLaunch + 1];
    int n_views;
    ViewsQueue *queue;
    float bg[3];
    float *rgb_out;
};

// Descriptors of the scene table reach the device the same way.
constexpr int kSetupItems = 24;

struct SceneSetupArgs {
    GridDev g[kSetupItems];
    int first, count, n_scenes, sh_dtype;
    SceneTableHeader *table;
    GridDev *scenes;
};

__global__ void scene_setup_kernel(SceneSetupArgs a) {
    const int i = threadIdx.x;
    if (i < a.count) a.scenes[a.first + i] = a.g[i];
    if (a.first == 0 && i == 0) {
        a.table->magic = kSceneMagic;
        a.table->n_scenes = a.n_scenes;
        a.table->sh_dtype = a.sh_dtype;
    }
}

// Persistent tile queue over all pixels of all views of the launch: each
// block takes the next 16x16-pixel tile, finds its view, generates the rays
// of its pixels (one per lane) and runs the same forward march as
// plx_render_fwd.  A pixel's colour depends only on its own ray and scene,
// never on the rest of the batch.
template <int DT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
void views_kernel(ViewsArgs a) {
    __shared__ long long tile_sh;
    // a table of other scenes' storage type (or not a scene table): nothing
    // is rendered and the status word says so
    const unsigned magic = a.table->magic;
    const int n_scenes = a.table->n_scenes, table_dt = a.table->sh_dtype;
    const bool ok = magic == kSceneMagic && table_dt == DT;
    if (!ok && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&a.queue->status, 1u);
    const int64_t n_tiles = ok ? a.tile_start[a.n_views] : 0;
    while (n_tiles > 0) {
        if (threadIdx.x == 0) tile_sh = (long long)atomicAdd(&a.queue->next, 1ull);
        __syncthreads();
        const int64_t tile = uni64(tile_sh);
        __syncthreads();
        if (tile >= n_tiles) break;
        int lo = 0;  // the view of the tile
        for (int i = 1; i < a.n_views; ++i)
            if (a.tile_start[i] <= tile) lo = i;
        const plx_view &v = a.v[lo];
        const int width = uni(v.width), height = uni(v.height);
        const int64_t tl = tile - a.tile_start[lo];
        const int tpr = (width + kTileW - 1) / kTileW;
        const int px = (int)(tl % tpr) * kTileW + (int)(threadIdx.x % kTileW);
        const int py = (int)(tl / tpr) * kTileH + (int)(threadIdx.x / kTileW);
        const int scene = uni(v.scene);
        if (scene >= n_scenes) {
            if (threadIdx.x == 0) atomicOr(&a.queue->status, 1u);
            continue;
        }
        if (px < width && py < height) {
            const GridDev g = uniform_grid(a.scenes[scene]);
            float o[3], d[3];
            camera_ray(v, px, py, o, d);
            RayGeom r;
            const int n = ray_setup(g, o, d, r);
            float y[9];
            sh_basis_all(d, y);
            CornerCache cc;
            cc.cell[0] = cc.cell[1] = cc.cell[2] = -1;
            float C[3];
            double tau;
            march_forward<DT>(g, r, n, y, cc, C, tau);
            const float T_final = expf(-(float)tau);
            float *out = a.rgb_out + 3 * (uni64(v.out_offset) + (int64_t)py * width + px);
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) out[c3] = C[c3] + T_final * a.bg[c3];
        }
    }
    // leave; the last block resets the queue for the next launch (every
    // block's last take from it precedes its leaving)
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.queue->done, 1u) == gridDim.x - 1) {
            atomicExch(&a.queue->next, 0ull);
            atomicExch(&a.queue->done, 0u);
        }
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
        for (int k = 0; k < n; ++k) {
            const Sample s = sample_at(g, r, k);
            const int64_t lin = cell_id(g, s.cell);
            if (!cell_occupied(g, s.cell)) continue;
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

template <int MODE, bool STATE = false>
int launch_render(const plx_grid *grid, RenderArgs &a, hipStream_t s, const char *fn) {
    const int64_t nb = (a.n_rays + kThreads - 1) / kThreads;
    if (nb > 0x7ffffff0) return fail(PLX_EINVAL, "%s: too many rays", fn);
    a.n_blocks = (int)nb;
    a.nb8 = round_up8(nb);
    GridDev g = to_dev(grid);
    if constexpr (MODE == MODE_FWD) {
        PLX_DISPATCH_DT(grid->sh_dtype, DT,
                        render_fwd_kernel<DT, STATE><<<a.nb8, kThreads, 0, s>>>(g, a));
    } else {
        static_assert(MODE == MODE_BWD, "the ray-order backward serves plx_render_bwd_state");
        PLX_DISPATCH_DT(grid->sh_dtype, DT, render_bwd_kernel<DT, STATE><<<a.nb8, kThreads, 0, s>>>(g, a));
    }
    return check_launch(fn);
}

// Layout of the per-sample state buffer: per-ray counts, then sample indices,
// then float4 values, each part 256-byte aligned.
struct StateLayout {
    int64_t kidx, vals, bytes;
};

StateLayout state_layout(int64_t n_rays, int32_t cap) {
    auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
    StateLayout l;
    l.kidx = up(n_rays * 4);
    l.vals = l.kidx + up(n_rays * (int64_t)cap * 4);
    l.bytes = l.vals + n_rays * (int64_t)cap * 16;
    return l;
}

int attach_state(RenderArgs &a, void *state, int64_t state_bytes, int32_t cap, const char *fn) {
    if (!state) return fail(PLX_EINVAL, "%s: state is NULL", fn);
    if (cap < 0 || cap > (1 << 20)) return fail(PLX_EINVAL, "%s: cap %d out of range", fn, (int)cap);
    if (reinterpret_cast<uintptr_t>(state) % 256)
        return fail(PLX_EINVAL, "%s: state must be 256-byte aligned", fn);
    const StateLayout l = state_layout(a.n_rays, cap);
    if (state_bytes < l.bytes)
        return fail(PLX_EINVAL, "%s: state of %lld bytes, need %lld", fn, (long long)state_bytes,
                    (long long)l.bytes);
    char *base = static_cast<char *>(state);
    a.st_count = reinterpret_cast<int *>(base);
    a.st_kidx = reinterpret_cast<int *>(base + l.kidx);
    a.st_vals = reinterpret_cast<float4 *>(base + l.vals);
    a.st_cap = cap;
    return PLX_OK;
}

// Exclusive scan of n counts into out[0..n] (out[n] = total).  tmp: 2*nb+1
// int64 where nb = ceil(n / kScanTile).
int scan_counts(const unsigned *c, int64_t n, int64_t *out, int64_t *tmp, hipStream_t s,
                const char *fn, int stride = 1) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb < 1 || nb > 0x7fffffff) return fail(PLX_EINVAL, "%s: bad scan size", fn);
    int64_t *bsum = tmp, *boff = tmp + nb;
    count_sum_kernel<<<(unsigned)nb, kScanT, 0, s>>>(c, n, stride, bsum);
    int rc = check_launch(fn);
    if (rc) return rc;
    block_offsets_kernel<<<1, kScanT, 0, s>>>(bsum, nb, boff);
    if ((rc = check_launch(fn))) return rc;
    count_scan_kernel<<<(unsigned)nb, kScanT, 0, s>>>(c, n, stride, boff, out);
    return check_launch(fn);
}

inline int64_t scan_tmp_words(int64_t n) { return 2 * ((n + kScanTile - 1) / kScanTile) + 1; }
inline int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// ------------------------------------------------------------ caller-owned bins
//
// The work lists of a batch live in two caller-owned buffers (plx_bins):
// the ray buffer holds the per-ray segment counts and offsets, the per-bin
// counts, cursors and offsets, the scan temporaries and a status word; the
// segment buffer holds the bin-major segment records and the per-segment
// values the render passes hand from one kernel to the next.

struct RayBufLayout {
    int64_t nseg, segoff, gray, bcount, bcursor, status, boff, scan;
    // per-bin sample counts (samples == true only)
    int64_t nbrick, bsoff, blist;
    int64_t bytes;
    bool samples;
};

// samples: with the per-bin sample counts and the brick list that the
// recorded backward needs (every caller-owned ray buffer has them; the
// fixed scratch of plx_render_train_static does not).
RayBufLayout ray_buf_layout(int64_t n_rays, int64_t nbk, bool samples = true) {
    RayBufLayout l = {};
    l.samples = samples;
    int64_t off = 0;
    l.nseg = off; off += align256(n_rays * 4);
    l.segoff = off; off += align256((n_rays + 1) * 8);
    l.gray = off; off += align256(n_rays * 16);
    // bin counts, cursors and the status word are cleared by one launch
    if (samples) {
        // 64-bit (segments, sample slots) counters and cursors, the status
        // word and the brick counter, cleared by one launch
        l.bcount = off; off += nbk * 8;
        l.bcursor = off; off += nbk * 8;
        l.status = off; off += 4;
        l.nbrick = off; off = align256(off + 4);
    } else {
        l.bcount = off; off += nbk * 4;
        l.bcursor = off; off += nbk * 4;
        l.status = off; off += align256(2 * nbk * 4 + 4) - 2 * nbk * 4;
    }
    l.boff = off; off += align256((nbk + 1) * 8);
    if (samples) {
        l.bsoff = off; off += align256((nbk + 1) * 8);
        l.blist = off; off += align256(nbk / kLenClasses * 4);
    }
    l.scan = off; off += align256((scan_tmp_words(n_rays) + scan_tmp_words(nbk)) * 8);
    l.bytes = off;
    return l;
}

struct SampBufLayout {
    int64_t soff, nocc, srec, bytes;
};

SampBufLayout samp_buf_layout(int64_t n_seg, int64_t n_samp) {
    SampBufLayout l;
    int64_t off = 0;
    l.soff = off; off += align256(n_seg * 8);
    l.nocc = off; off += align256(n_seg * 4);
    l.srec = off; off += align256(n_samp * (int64_t)sizeof(SampleRec));
    l.bytes = off;
    return l;
}

// Sample slots one call handles (the scatter numbers a pass's samples with
// 32-bit integers; the records are addressed with 64-bit offsets).
constexpr int64_t kMaxSampBinned = (int64_t)1 << 40;

struct SegBufLayout {
    int64_t bseg, tseg, cseg, tin, gra, bytes;
};

SegBufLayout seg_buf_layout(int64_t n_seg) {
    SegBufLayout l;
    int64_t off = 0;
    l.bseg = off; off += align256(n_seg * 16);
    l.tseg = off; off += align256(n_seg * 8);
    l.cseg = off; off += align256(n_seg * 16);
    l.tin = off; off += align256(n_seg * 8);
    l.gra = off; off += align256(n_seg * 4);
    l.bytes = off;
    return l;
}

constexpr int64_t kMaxRaysBinned = 0x7fffffffLL - kThreads;

// Points a's per-ray and per-bin arrays into a ray buffer.
void attach_ray_buf(BinArgs &a, void *ray_buf, const RayBufLayout &l) {
    char *base = static_cast<char *>(ray_buf);
    a.nseg = reinterpret_cast<unsigned *>(base + l.nseg);
    a.seg_off = reinterpret_cast<int64_t *>(base + l.segoff);
    a.g_ray = reinterpret_cast<float4 *>(base + l.gray);
    a.status = reinterpret_cast<unsigned *>(base + l.status);
    a.boff = reinterpret_cast<int64_t *>(base + l.boff);
    if (l.samples) {
        a.bcnt64 = reinterpret_cast<unsigned long long *>(base + l.bcount);
        a.bcur64 = reinterpret_cast<unsigned long long *>(base + l.bcursor);
        a.bcount = reinterpret_cast<unsigned *>(base + l.bcount);  // the low halves, read at stride 2
        a.nbrick = reinterpret_cast<unsigned *>(base + l.nbrick);
        a.bsoff = reinterpret_cast<int64_t *>(base + l.bsoff);
        a.blist = reinterpret_cast<unsigned *>(base + l.blist);
    } else {
        a.bcount = reinterpret_cast<unsigned *>(base + l.bcount);
        a.bcursor = reinterpret_cast<unsigned *>(base + l.bcursor);
    }
}

// Points a's recorded-backward arrays into a sample buffer.
void attach_samp_buf(BinArgs &a, void *samp_buf, const SampBufLayout &l) {
    char *b = static_cast<char *>(samp_buf);
    a.soff = reinterpret_cast<int64_t *>(b + l.soff);
    a.nocc = reinterpret_cast<int *>(b + l.nocc);
    a.srec = reinterpret_cast<SampleRec *>(b + l.srec);
}

// Points a's per-segment arrays into a segment buffer.
void attach_seg_buf(BinArgs &a, void *seg_buf, const SegBufLayout &l) {
    char *b2 = static_cast<char *>(seg_buf);
    a.bseg = reinterpret_cast<int4 *>(b2 + l.bseg);
    a.tau_seg = reinterpret_cast<double *>(b2 + l.tseg);
    a.c_seg = reinterpret_cast<float4 *>(b2 + l.cseg);
    a.tau_in = reinterpret_cast<double *>(b2 + l.tin);
    a.gr_after = reinterpret_cast<float *>(b2 + l.gra);
}

int check_buf(const void *p, int64_t have, int64_t need, const char *what, const char *fn) {
    if (!p) return fail(PLX_EINVAL, "%s: %s is NULL", fn, what);
    if (reinterpret_cast<uintptr_t>(p) % 256) return fail(PLX_EINVAL, "%s: %s must be 256-byte aligned", fn, what);
    if (have < need)
        return fail(PLX_EINVAL, "%s: %s of %lld bytes, need %lld", fn, what, (long long)have, (long long)need);
    return PLX_OK;
}

// Validates bins against the grid and batch of a render call and points a's
// arrays into them.
int attach_bins(const plx_grid *grid, const plx_bins *bins, int64_t n_rays, BinArgs &a, const char *fn) {
    if (!bins) return fail(PLX_EINVAL, "%s: bins is NULL", fn);
    if (bins->n_rays != n_rays)
        return fail(PLX_EINVAL, "%s: bins were made for %lld rays, the call has %lld", fn,
                    (long long)bins->n_rays, (long long)n_rays);
    if (bins->n_seg < 0 || bins->n_seg > kMaxRaysBinned)
        return fail(PLX_EINVAL, "%s: bins->n_seg = %lld out of range", fn, (long long)bins->n_seg);
    const RayBufLayout rl = ray_buf_layout(n_rays, n_bins(to_dev(grid)));
    int rc = check_buf(bins->ray_buf, bins->ray_buf_bytes, rl.bytes, "bins->ray_buf", fn);
    if (rc) return rc;
    attach_ray_buf(a, bins->ray_buf, rl);
    a.n_seg = bins->n_seg;
    a.seg_cap = bins->n_seg;
    if (bins->n_seg > 0) {
        const SegBufLayout sl = seg_buf_layout(bins->n_seg);
        if ((rc = check_buf(bins->seg_buf, bins->seg_buf_bytes, sl.bytes, "bins->seg_buf", fn))) return rc;
        attach_seg_buf(a, bins->seg_buf, sl);
    }
    const int64_t n_bricks = n_bins(to_dev(grid)) / kLenClasses;
    if (bins->n_brick < 0 || bins->n_brick > n_bricks || (bins->n_seg > 0) != (bins->n_brick > 0))
        return fail(PLX_EINVAL, "%s: bins->n_brick = %lld out of range", fn, (long long)bins->n_brick);
    if (bins->n_samp < 0 || bins->n_samp > kMaxSampBinned || (bins->n_seg > 0 && bins->n_samp < bins->n_seg))
        return fail(PLX_EINVAL, "%s: bins->n_samp = %lld out of range", fn, (long long)bins->n_samp);
    a.n_brick = bins->n_brick;
    if (bins->samp_buf && bins->n_seg > 0) {
        const SampBufLayout pl = samp_buf_layout(bins->n_seg, bins->n_samp);
        if ((rc = check_buf(bins->samp_buf, bins->samp_buf_bytes, pl.bytes, "bins->samp_buf", fn))) return rc;
        attach_samp_buf(a, bins->samp_buf, pl);
        a.samp_cap = bins->n_samp;
    }
    return PLX_OK;
}

// Counting phase: per-ray and per-bin segment counts and their scans.
// Leaves the total at seg_off[n_rays] on the device.
int bin_count_launch(const GridDev &g, BinArgs &a, int64_t nbk, int64_t *scan_tmp, hipStream_t s,
                     const char *fn) {
    const int64_t n_rays = a.n_rays;
    // counters, cursors, the status word (and the brick counter)
    const int64_t nz = a.bcnt64 ? 4 * nbk + 2 : 2 * nbk + 1;
    zero_u32_kernel<<<(unsigned)((nz + 255) / 256), 256, 0, s>>>(
        a.bcnt64 ? reinterpret_cast<unsigned *>(a.bcnt64) : a.bcount, nz);
    int rc = check_launch(fn);
    if (rc) return rc;
    const int64_t nbr = (n_rays + kThreads - 1) / kThreads;
    a.n_blocks = (int)nbr;
    a.nb8 = round_up8(nbr);
    seg_count_kernel<<<a.nb8, kThreads, 0, s>>>(g, a);
    if ((rc = check_launch(fn))) return rc;
    if ((rc = scan_counts(a.nseg, n_rays, a.seg_off, scan_tmp, s, fn))) return rc;
    int64_t *bin_tmp = scan_tmp + scan_tmp_words(n_rays);
    if (!a.bcnt64) return scan_counts(a.bcount, nbk, a.boff, bin_tmp, s, fn);
    const unsigned *halves = reinterpret_cast<const unsigned *>(a.bcnt64);
    if ((rc = scan_counts(halves, nbk, a.boff, bin_tmp, s, fn, 2))) return rc;
    if ((rc = scan_counts(halves + 1, nbk, a.bsoff, bin_tmp, s, fn, 2))) return rc;
    const int64_t n_bricks = nbk / kLenClasses;
    brick_list_kernel<<<(unsigned)((n_bricks + kThreads - 1) / kThreads), kThreads, 0, s>>>(a, n_bricks);
    return check_launch(fn);
}

// Render passes over binned segments: MODE_FWD renders, MODE_BWD and
// MODE_TRAIN also run the backward replay, MODE_MAXW the weight passes.
// Launch sizes come from a.n_seg, an upper bound when a.n_seg_dev is set.
// Records the caller's timing event i (when given) on the stream.
int mark_event(void **events, int i, hipStream_t s, const char *fn) {
    if (!events || !events[i]) return PLX_OK;
    PLX_CHECK_HIP(hipEventRecord(static_cast<hipEvent_t>(events[i]), s), fn);
    return PLX_OK;
}

template <int MODE>
int render_binned(const plx_grid *grid, BinArgs a, hipStream_t s, const char *fn) {
    GridDev g = to_dev(grid);
    const int64_t nbr = (a.n_rays + kThreads - 1) / kThreads;
    const int64_t nbs = (a.n_seg + kThreads - 1) / kThreads;
    BinArgs as = a;
    as.n_blocks = (int)nbs;
    as.nb8 = round_up8(nbs);
    int rc;
    if ((rc = mark_event(a.events, 0, s, fn))) return rc;
    if constexpr (MODE == MODE_MAXW) {
        if (a.n_seg == 0) return PLX_OK;
        PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_weight_kernel<DT, 0><<<as.nb8, kThreads, 0, s>>>(g, as));
        if ((rc = check_launch(fn))) return rc;
        seg_combine_kernel<MODE><<<(unsigned)nbr, kThreads, 0, s>>>(a);
        if ((rc = check_launch(fn))) return rc;
        PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_weight_kernel<DT, 1><<<as.nb8, kThreads, 0, s>>>(g, as));
        return check_launch(fn);
    }
    if (a.n_seg > 0) {
        const bool rec = MODE != MODE_FWD && a.srec;
        const bool lists = a.blist && a.n_brick > 0;
        if (rec && lists && a.n_seg >= kFwdParMinSegs * a.n_brick) {
            // recording forward: sample-parallel, one workgroup per brick
            PLX_DISPATCH_DT(grid->sh_dtype, DT,
                            seg_fwd_samples_kernel<DT><<<(unsigned)a.n_brick, kFwdThreads, 0, s>>>(g, as));
        } else if (lists && grid->sh_dtype != PLX_F32) {
            // brick-staged (16-bit records: 47 KB of LDS per brick, three
            // workgroups per CU; FP32's 82 KB leave one, and the lane-per-
            // segment kernel with its L2 traffic is then twice as fast)
            const unsigned nb = (unsigned)a.n_brick;
            if (rec) {
                PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_fwd_brick_kernel<DT, true><<<nb, kThreads, 0, s>>>(g, as));
            } else {
                PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_fwd_brick_kernel<DT, false><<<nb, kThreads, 0, s>>>(g, as));
            }
        } else if (rec) {
            PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_fwd_kernel<DT, true><<<as.nb8, kThreads, 0, s>>>(g, as));
        } else {
            PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_fwd_kernel<DT, false><<<as.nb8, kThreads, 0, s>>>(g, as));
        }
        if ((rc = check_launch(fn))) return rc;
    }
    if ((rc = mark_event(a.events, 1, s, fn))) return rc;
    seg_combine_kernel<MODE><<<(unsigned)nbr, kThreads, 0, s>>>(a);
    if ((rc = check_launch(fn))) return rc;
    if ((rc = mark_event(a.events, 2, s, fn))) return rc;
    if (MODE != MODE_FWD && a.n_seg > 0 && a.srec) {
        // recorded backward: one scatter workgroup per brick (the Cauchy
        // prior's per-sample terms only in an instance of their own)
        if (a.n_brick > 0) {
            if (as.pri.lambda_s != 0.0f)
                seg_scatter_kernel<true><<<(unsigned)a.n_brick, kScatterThreads, 0, s>>>(g, as);
            else
                seg_scatter_kernel<false><<<(unsigned)a.n_brick, kScatterThreads, 0, s>>>(g, as);
            if ((rc = check_launch(fn))) return rc;
        }
    } else if (MODE != MODE_FWD && a.n_seg > 0) {
        // the Cauchy prior's per-sample terms only in an instance of their own
        if (as.pri.lambda_s != 0.0f) {
            PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_bwd_kernel<DT, true><<<as.nb8, kThreads, 0, s>>>(g, as));
        } else {
            PLX_DISPATCH_DT(grid->sh_dtype, DT, seg_bwd_kernel<DT, false><<<as.nb8, kThreads, 0, s>>>(g, as));
        }
        if ((rc = check_launch(fn))) return rc;
    }
    return mark_event(a.events, 3, s, fn);
}

// Priors of a gradient call from its options (validated).
int priors_from(const plx_render_opts *opts, Priors &p, const char *fn) {
    p.lambda_s = opts->lambda_sparsity;
    p.lambda_b = opts->lambda_beta;
    p.eps = opts->beta_eps;
    p.loss = opts->reg_loss_sum;
    if (!std::isfinite(p.lambda_s) || !std::isfinite(p.lambda_b))
        return fail(PLX_EINVAL, "%s: prior weights must be finite", fn);
    if (p.lambda_b != 0.0f && !(p.eps > 0.0f && std::isfinite(p.eps)))
        return fail(PLX_EINVAL, "%s: beta_eps must be > 0 when lambda_beta != 0", fn);
    return PLX_OK;
}

RenderArgs base_args(const plx_render_opts *opts, const float *o, const float *d, int64_t n) {
    RenderArgs a = {};
    a.rays_o = o;
    a.rays_d = d;
    a.n_rays = n;
    for (int i = 0; i < 3; ++i) a.bg[i] = opts->background[i];
    a.bg_rgb = opts->background_rgb;
    a.grad_bg = opts->grad_background;
    return a;
}

// ------------------------------------------------------------ fixed scratch
//
// plx_render_train_static serves callers that cannot allocate (code under
// graph capture, serving loops): its segment lists live in a fixed device
// array instead of caller buffers, sized for the worst case of the batch
// (every ray crossing the most bricks a line can cross), and the segment
// kernels read the true segment count on the device, so the call neither
// allocates nor synchronises.  The array is per device and kept until the
// process ends; calls that overlap on one device share it and race.
constexpr int64_t kStaticScratchBytes = (int64_t)64 << 20;
constexpr int kMaxDevices = 64;

std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Device address of this device's fixed scratch, looked up once per device
// (the array's name is a host-side stand-in, never passed to a kernel).
int static_scratch(void **out, const char *fn) {
    int dev = 0;
    PLX_CHECK_HIP(hipGetDevice(&dev), fn);
    if (dev < 0 || dev >= kMaxDevices) return fail(PLX_EDEVICE, "%s: device %d out of range", fn, dev);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        PLX_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), fn);
        if (!p) return fail(PLX_EDEVICE, "%s: no address for the fixed scratch", fn);
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return PLX_OK;
}

}  // namespace
}  // namespace plx

using namespace plx;

extern "C" {

int64_t plx_bins_ray_bytes(const int32_t reso[3], int64_t n_rays) {
    if (!reso || reso[0] < 2 || reso[1] < 2 || reso[2] < 2 || n_rays < 0 || n_rays > kMaxRaysBinned)
        return 0;
    plx_grid tmp = {};
    for (int a = 0; a < 3; ++a) tmp.reso[a] = reso[a];
    return ray_buf_layout(n_rays, n_bins(to_dev(&tmp))).bytes;
}

int64_t plx_bins_seg_bytes(int64_t n_seg) {
    if (n_seg < 0 || n_seg > kMaxRaysBinned) return 0;
    return seg_buf_layout(n_seg).bytes;
}

int64_t plx_bins_samp_bytes(int64_t n_seg, int64_t n_samp) {
    if (n_seg < 0 || n_seg > kMaxRaysBinned || n_samp < 0 || n_samp > kMaxSampBinned) return 0;
    return samp_buf_layout(n_seg, n_samp).bytes;
}

int plx_bins_count(const plx_grid *grid, const float *rays_o, const float *rays_d, int64_t n_rays,
                   void *ray_buf, int64_t ray_buf_bytes, plx_bins *bins, plx_stream stream) {
    const char *fn = "plx_bins_count";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!bins) return fail(PLX_EINVAL, "%s: bins is NULL", fn);
    if (n_rays > kMaxRaysBinned) return fail(PLX_EINVAL, "%s: too many rays", fn);
    const GridDev g = to_dev(grid);
    const int64_t nbk = n_bins(g);
    const RayBufLayout l = ray_buf_layout(n_rays, nbk);
    if ((rc = check_buf(ray_buf, ray_buf_bytes, l.bytes, "ray_buf", fn))) return rc;
    *bins = plx_bins{};
    bins->n_rays = n_rays;
    bins->ray_buf = ray_buf;
    bins->ray_buf_bytes = ray_buf_bytes;
    if (n_rays == 0) return PLX_OK;
    hipStream_t s = as_stream(stream);
    BinArgs a = {};
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.n_rays = n_rays;
    attach_ray_buf(a, ray_buf, l);
    int64_t *scan_tmp = reinterpret_cast<int64_t *>(static_cast<char *>(ray_buf) + l.scan);
    if ((rc = bin_count_launch(g, a, nbk, scan_tmp, s, fn))) return rc;
    int64_t total = 0, samples = 0;
    unsigned bricks = 0;
    PLX_CHECK_HIP(hipMemcpyAsync(&total, a.seg_off + n_rays, sizeof(total), hipMemcpyDeviceToHost, s), fn);
    PLX_CHECK_HIP(hipMemcpyAsync(&samples, a.bsoff + nbk, sizeof(samples), hipMemcpyDeviceToHost, s), fn);
    PLX_CHECK_HIP(hipMemcpyAsync(&bricks, a.nbrick, sizeof(bricks), hipMemcpyDeviceToHost, s), fn);
    PLX_CHECK_HIP(hipStreamSynchronize(s), fn);
    if (total < 0 || total > kMaxRaysBinned)
        return fail(PLX_EINVAL, "%s: %lld ray segments, more than one call handles", fn, (long long)total);
    if (samples < 0 || samples > kMaxSampBinned)
        return fail(PLX_EINVAL, "%s: %lld sample slots, more than one call handles", fn, (long long)samples);
    bins->n_seg = total;
    bins->n_samp = samples;
    bins->n_brick = bricks;
    return PLX_OK;
}

int plx_bins_apply(const plx_grid *grid, const float *rays_o, const float *rays_d,
                   const plx_bins *bins, plx_stream stream) {
    const char *fn = "plx_bins_apply";
    int rc = validate_grid(grid, true, fn);
    if (rc) return rc;
    if (!bins) return fail(PLX_EINVAL, "%s: bins is NULL", fn);
    if ((rc = validate_rays(rays_o, rays_d, bins->n_rays, fn))) return rc;
    BinArgs a = {};
    if ((rc = attach_bins(grid, bins, bins->n_rays, a, fn))) return rc;
    if (bins->n_seg == 0) return PLX_OK;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.n_rays = bins->n_rays;
    const int64_t nbr = (a.n_rays + kThreads - 1) / kThreads;
    a.n_blocks = (int)nbr;
    a.nb8 = round_up8(nbr);
    seg_emit_kernel<<<a.nb8, kThreads, 0, as_stream(stream)>>>(to_dev(grid), a);
    return check_launch(fn);
}

int plx_bins_verify(const plx_grid *grid, const plx_bins *bins, plx_stream stream) {
    const char *fn = "plx_bins_verify";
    int rc = validate_grid(grid, true, fn);
    if (rc) return rc;
    BinArgs a = {};
    if (!bins) return fail(PLX_EINVAL, "%s: bins is NULL", fn);
    if ((rc = attach_bins(grid, bins, bins->n_rays, a, fn))) return rc;
    if (bins->n_rays == 0) return PLX_OK;
    hipStream_t s = as_stream(stream);
    unsigned st = 0;
    PLX_CHECK_HIP(hipMemcpyAsync(&st, a.status, sizeof(st), hipMemcpyDeviceToHost, s), fn);
    PLX_CHECK_HIP(hipStreamSynchronize(s), fn);
    if (st != 0) return fail(PLX_EDEVICE, "%s: the segment walk of plx_bins_apply disagreed with plx_bins_count", fn);
    return PLX_OK;
}

int plx_render_fwd(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                   const float *rays_d, int64_t n_rays, const plx_bins *bins, float *rgb_out,
                   float *tau_out, plx_stream stream) {
    const char *fn = "plx_render_fwd";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!rgb_out) return fail(PLX_EINVAL, "%s: rgb_out is NULL", fn);
    BinArgs a = {};
    if ((rc = attach_bins(grid, bins, n_rays, a, fn))) return rc;
    a.events = opts->kernel_events;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.rgb_out = rgb_out;
    a.tau_out = tau_out;
    a.n_rays = n_rays;
    for (int i = 0; i < 3; ++i) a.bg[i] = opts->background[i];
    a.bg_rgb = opts->background_rgb;
    a.grad_bg = opts->grad_background;
    return render_binned<MODE_FWD>(grid, a, as_stream(stream), fn);
}

int plx_render_bwd(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                   const float *rays_d, int64_t n_rays, const plx_bins *bins, const float *grad_rgb,
                   const float *tau_fwd, float *grad, uint8_t *touched, plx_stream stream) {
    const char *fn = "plx_render_bwd";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!grad_rgb || !tau_fwd || (grid->n_vox > 0 && (!grad || !touched)))
        return fail(PLX_EINVAL, "%s: NULL grad_rgb/tau_fwd/grad/touched", fn);
    BinArgs a = {};
    if ((rc = priors_from(opts, a.pri, fn))) return rc;
    if ((rc = attach_bins(grid, bins, n_rays, a, fn))) return rc;
    a.events = opts->kernel_events;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.grad_rgb = grad_rgb;
    a.grad = grad;
    a.touched = touched;
    a.n_rays = n_rays;
    for (int i = 0; i < 3; ++i) a.bg[i] = opts->background[i];
    a.bg_rgb = opts->background_rgb;
    a.grad_bg = opts->grad_background;
    return render_binned<MODE_BWD>(grid, a, as_stream(stream), fn);
}

int plx_render_max_weight(const plx_grid *grid, const float *rays_o, const float *rays_d,
                          int64_t n_rays, const plx_bins *bins, float *wmax, plx_stream stream) {
    const char *fn = "plx_render_max_weight";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (n_rays == 0) return PLX_OK;
    if (!wmax) return fail(PLX_EINVAL, "%s: wmax is NULL", fn);
    BinArgs a = {};
    if ((rc = attach_bins(grid, bins, n_rays, a, fn))) return rc;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.wmax = wmax;
    a.n_rays = n_rays;
    return render_binned<MODE_MAXW>(grid, a, as_stream(stream), fn);
}

int plx_render_train(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                     const float *rays_d, const float *target, int64_t n_rays, const plx_bins *bins,
                     float loss_scale, float *rgb_out, float *grad, uint8_t *touched,
                     double *loss_sum, plx_stream stream) {
    const char *fn = "plx_render_train";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!target || !loss_sum || (grid->n_vox > 0 && (!grad || !touched)))
        return fail(PLX_EINVAL, "%s: NULL target/grad/touched/loss_sum", fn);
    BinArgs a = {};
    if ((rc = priors_from(opts, a.pri, fn))) return rc;
    if ((rc = attach_bins(grid, bins, n_rays, a, fn))) return rc;
    a.events = opts->kernel_events;
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.target = target;
    a.rgb_out = rgb_out;
    a.loss_sum = loss_sum;
    a.grad = grad;
    a.touched = touched;
    a.n_rays = n_rays;
    for (int i = 0; i < 3; ++i) a.bg[i] = opts->background[i];
    a.bg_rgb = opts->background_rgb;
    a.grad_bg = opts->grad_background;
    a.loss_scale = loss_scale;
    return render_binned<MODE_TRAIN>(grid, a, as_stream(stream), fn);
}

int plx_render_train_static(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                            const float *rays_d, const float *target, int64_t n_rays,
                            float loss_scale, float *rgb_out, float *grad, uint8_t *touched,
                            double *loss_sum, plx_stream stream) {
    const char *fn = "plx_render_train_static";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!target || !loss_sum || (grid->n_vox > 0 && (!grad || !touched)))
        return fail(PLX_EINVAL, "%s: NULL target/grad/touched/loss_sum", fn);
    const GridDev g = to_dev(grid);
    const int64_t nbk = n_bins(g);
    // a ray enters each brick at most once and a line crosses at most
    // bx + by + bz - 2 bricks of the lattice
    const int64_t per_ray = (int64_t)g.bx + g.by + g.bz;
    const int64_t cap = n_rays * per_ray;
    const RayBufLayout rl = ray_buf_layout(n_rays, nbk, false);
    const SegBufLayout sl = seg_buf_layout(cap);
    if (n_rays > kMaxRaysBinned || cap > kMaxRaysBinned || rl.bytes + sl.bytes > kStaticScratchBytes)
        return fail(PLX_ENOMEM,
                    "%s: %lld rays on a %dx%dx%d grid need %lld bytes of scratch, more than the fixed %lld "
                    "(the bound is ray buffer + %lld segments per ray)",
                    fn, (long long)n_rays, grid->reso[0], grid->reso[1], grid->reso[2],
                    (long long)(rl.bytes + sl.bytes), (long long)kStaticScratchBytes, (long long)per_ray);
    BinArgs a = {};
    if ((rc = priors_from(opts, a.pri, fn))) return rc;
    void *base = nullptr;
    if ((rc = static_scratch(&base, fn))) return rc;
    hipStream_t s = as_stream(stream);
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.n_rays = n_rays;
    attach_ray_buf(a, base, rl);
    attach_seg_buf(a, static_cast<char *>(base) + rl.bytes, sl);
    int64_t *scan_tmp = reinterpret_cast<int64_t *>(static_cast<char *>(base) + rl.scan);
    // counts, scans and records: the previous call's contents are cleared
    // by the counting phase (bin counters, cursors, status)
    if ((rc = bin_count_launch(g, a, nbk, scan_tmp, s, fn))) return rc;
    a.n_seg = cap;  // launch bound; the kernels read the count itself
    a.seg_cap = cap;
    a.n_seg_dev = a.seg_off + n_rays;
    seg_emit_kernel<<<a.nb8, kThreads, 0, s>>>(g, a);
    if ((rc = check_launch(fn))) return rc;
    a.events = opts->kernel_events;
    a.target = target;
    a.rgb_out = rgb_out;
    a.loss_sum = loss_sum;
    a.grad = grad;
    a.touched = touched;
    for (int i = 0; i < 3; ++i) a.bg[i] = opts->background[i];
    a.bg_rgb = opts->background_rgb;
    a.grad_bg = opts->grad_background;
    a.loss_scale = loss_scale;
    return render_binned<MODE_TRAIN>(grid, a, s, fn);
}

int64_t plx_render_state_bytes(int64_t n_rays, int32_t cap) {
    if (n_rays < 0 || cap < 0 || cap > (1 << 20)) return 0;
    return state_layout(n_rays, cap).bytes;
}

int plx_render_fwd_state(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                         const float *rays_d, int64_t n_rays, float *rgb_out, float *tau_out,
                         void *state, int64_t state_bytes, int32_t cap, plx_stream stream) {
    const char *fn = "plx_render_fwd_state";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!rgb_out) return fail(PLX_EINVAL, "%s: rgb_out is NULL", fn);
    RenderArgs a = base_args(opts, rays_o, rays_d, n_rays);
    if ((rc = attach_state(a, state, state_bytes, cap, fn))) return rc;
    a.rgb_out = rgb_out;
    a.tau_out = tau_out;
    return launch_render<MODE_FWD, true>(grid, a, as_stream(stream), fn);
}

int plx_render_bwd_state(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                         const float *rays_d, int64_t n_rays, const float *grad_rgb,
                         const float *tau_fwd, const void *state, int64_t state_bytes, int32_t cap,
                         float *grad, uint8_t *touched, plx_stream stream) {
    const char *fn = "plx_render_bwd_state";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_rays == 0) return PLX_OK;
    if (!grad_rgb || !tau_fwd || (grid->n_vox > 0 && (!grad || !touched)))
        return fail(PLX_EINVAL, "%s: NULL grad_rgb/tau_fwd/grad/touched", fn);
    RenderArgs a = base_args(opts, rays_o, rays_d, n_rays);
    if ((rc = priors_from(opts, a.pri, fn))) return rc;
    if ((rc = attach_state(a, const_cast<void *>(state), state_bytes, cap, fn))) return rc;
    a.grad_rgb = grad_rgb;
    a.tau_in = tau_fwd;
    a.grad = grad;
    a.touched = touched;
    return launch_render<MODE_BWD, true>(grid, a, as_stream(stream), fn);
}

int64_t plx_scene_table_bytes(int32_t n_scenes) {
    if (n_scenes < 1) return 0;
    return kSceneTableHead + (int64_t)n_scenes * (int64_t)sizeof(GridDev);
}

int plx_scene_table_set(const plx_grid *scenes, int32_t n_scenes, void *table, int64_t table_bytes,
                        plx_stream stream) {
    const char *fn = "plx_scene_table_set";
    if (!scenes || n_scenes < 1) return fail(PLX_EINVAL, "%s: need at least one scene", fn);
    if (!table || reinterpret_cast<uintptr_t>(table) % 256)
        return fail(PLX_EINVAL, "%s: table must be a 256-byte aligned device pointer", fn);
    if (table_bytes < plx_scene_table_bytes(n_scenes))
        return fail(PLX_EINVAL, "%s: table of %lld bytes, need %lld", fn, (long long)table_bytes,
                    (long long)plx_scene_table_bytes(n_scenes));
    const int32_t dt = scenes[0].sh_dtype;
    for (int32_t i = 0; i < n_scenes; ++i) {
        int rc = validate_grid(&scenes[i], true, fn);
        if (rc) return rc;
        if (scenes[i].sh_dtype != dt) return fail(PLX_EINVAL, "%s: scenes must share one sh_dtype", fn);
    }
    hipStream_t s = as_stream(stream);
    SceneSetupArgs a = {};
    a.n_scenes = n_scenes;
    a.sh_dtype = dt;
    a.table = static_cast<SceneTableHeader *>(table);
    a.scenes = reinterpret_cast<GridDev *>(static_cast<char *>(table) + kSceneTableHead);
    for (int32_t first = 0; first < n_scenes; first += kSetupItems) {
        a.first = first;
        a.count = std::min(kSetupItems, n_scenes - first);
        for (int i = 0; i < a.count; ++i) a.g[i] = to_dev(&scenes[first + i]);
        scene_setup_kernel<<<1, 32, 0, s>>>(a);
        int rc = check_launch(fn);
        if (rc) return rc;
    }
    return PLX_OK;
}

int plx_render_views(const void *scene_table, int32_t n_scenes, int32_t sh_dtype, const plx_view *views,
                     int32_t n_views, const plx_render_opts *opts, float *rgb_out, void *queue,
                     plx_stream stream) {
    const char *fn = "plx_render_views";
    if (!scene_table || n_scenes < 1) return fail(PLX_EINVAL, "%s: need a scene table of at least one scene", fn);
    if (sh_dtype != PLX_F32 && sh_dtype != PLX_BF16 && sh_dtype != PLX_F16)
        return fail(PLX_EINVAL, "%s: bad sh_dtype %d", fn, sh_dtype);
    if (n_views < 0) return fail(PLX_EINVAL, "%s: n_views < 0", fn);
    if (!opts) return fail(PLX_EINVAL, "%s: opts is NULL", fn);
    if (n_views == 0) return PLX_OK;
    if (!views || !rgb_out || !queue) return fail(PLX_EINVAL, "%s: NULL views/rgb_out/queue", fn);
    if (reinterpret_cast<uintptr_t>(queue) % 256)
        return fail(PLX_EINVAL, "%s: queue must be 256-byte aligned", fn);
    for (int32_t i = 0; i < n_views; ++i) {
        const plx_view &v = views[i];
        if (v.scene < 0 || v.scene >= n_scenes) return fail(PLX_EINVAL, "%s: view %d: bad scene", fn, i);
        if (v.width < 1 || v.height < 1 || v.width > 65536 || v.height > 65536)
            return fail(PLX_EINVAL, "%s: view %d: bad size %dx%d", fn, i, v.width, v.height);
        if (!(v.focal > 0.0) || !std::isfinite(v.focal) || v.out_offset < 0)
            return fail(PLX_EINVAL, "%s: view %d: bad focal or out_offset", fn, i);
    }
    hipStream_t s = as_stream(stream);
    ViewsArgs va;
    va.table = static_cast<const SceneTableHeader *>(scene_table);
    va.scenes = reinterpret_cast<const GridDev *>(static_cast<const char *>(scene_table) + kSceneTableHead);
    va.queue = static_cast<ViewsQueue *>(queue);
    va.rgb_out = rgb_out;
    for (int i = 0; i < 3; ++i) va.bg[i] = opts->background[i];
    for (int32_t first = 0; first < n_views; first += kViewsPerLaunch) {
        va.n_views = std::min(kViewsPerLaunch, n_views - first);
        int64_t tiles = 0;
        for (int i = 0; i < va.n_views; ++i) {
            const plx_view &v = views[first + i];
            va.v[i] = v;
            va.tile_start[i] = tiles;
            tiles += (int64_t)((v.width + kTileW - 1) / kTileW) * ((v.height + kTileH - 1) / kTileH);
        }
        va.tile_start[va.n_views] = tiles;
        const int64_t nblk = tiles < 2048 ? tiles : 2048;  // persistent: 8 blocks per CU
        PLX_DISPATCH_DT(sh_dtype, DT, views_kernel<DT><<<(unsigned)nblk, kThreads, 0, s>>>(va));
        int rc = check_launch(fn);
        if (rc) return rc;
    }
    return PLX_OK;
}

int plx_render_views_status(const void *queue, plx_stream stream) {
    const char *fn = "plx_render_views_status";
    if (!queue) return fail(PLX_EINVAL, "%s: queue is NULL", fn);
    hipStream_t s = as_stream(stream);
    unsigned st = 0;
    PLX_CHECK_HIP(hipMemcpyAsync(&st, &static_cast<const ViewsQueue *>(queue)->status, sizeof(st),
                                 hipMemcpyDeviceToHost, s), fn);
    PLX_CHECK_HIP(hipStreamSynchronize(s), fn);
    if (st != 0)
        return fail(PLX_EINVAL, "%s: a launch on this queue met a scene table of another storage type, or "
                                "a view naming a scene beyond it; those views were not rendered", fn);
    return PLX_OK;
}

int plx_render_stats(const plx_grid *grid, const float *rays_o, const float *rays_d,
                     int64_t n_rays, uint32_t *cell_mark, uint32_t *vox_mark, void *ws,
                     int64_t ws_bytes, int64_t counts[4], plx_stream stream) {
    const char *fn = "plx_render_stats";
    int rc = validate_grid(grid, true, fn);
    if (rc || (rc = validate_rays(rays_o, rays_d, n_rays, fn))) return rc;
    if (!cell_mark || !vox_mark || !counts) return fail(PLX_EINVAL, "%s: NULL argument", fn);
    if ((rc = check_buf(ws, ws_bytes, PLX_COUNT_WORKSPACE_BYTES, "workspace", fn))) return rc;
    hipStream_t s = as_stream(stream);
    const int64_t cw = (n_cells(grid->reso) + 31) / 32, vw = (grid->n_vox + 31) / 32;
    zero_u32_kernel<<<(unsigned)((cw + 255) / 256), 256, 0, s>>>(cell_mark, cw);
    if ((rc = check_launch(fn))) return rc;
    if (vw) {
        zero_u32_kernel<<<(unsigned)((vw + 255) / 256), 256, 0, s>>>(vox_mark, vw);
        if ((rc = check_launch(fn))) return rc;
    }
    // two sample counters at the start of the workspace (the bit counts
    // below reuse its first word after these are read back)
    auto *cnt = static_cast<unsigned long long *>(ws);
    zero_u32_kernel<<<1, 256, 0, s>>>(static_cast<unsigned *>(ws), 4);
    if ((rc = check_launch(fn))) return rc;
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
    if ((rc = count_set_bits(cell_mark, n_cells(grid->reso), ws, &cells, s, fn))) return rc;
    if ((rc = count_set_bits(vox_mark, grid->n_vox, ws, &vox, s, fn))) return rc;
    counts[2] = cells;
    counts[3] = vox;
    return PLX_OK;
}

}  // extern "C"
