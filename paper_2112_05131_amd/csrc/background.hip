// background.hip -- the multi-sphere (MSI) background model of 360-degree
// scenes (Sec. 3.6, background model; supplement B.1) for gfx950.
//
// The background is a grid of reso (L, H, W): L spheres around the origin,
// spaced linearly in inverse radius (grid coordinate u = (1 - 1/r) L - 1/2,
// sphere l at u = l), each an equirectangular image of H rows (polar angle
// from +z) and W columns (azimuth from +x towards +y).  Voxels hold an
// opacity density (record slot 28) and a degree-0 colour coefficient per
// channel (slots 24, 25, 26) in FP32 records; NULL reads as zero.  A ray's
// samples sit at u = k/2, k = 0 .. 2(L-1)-1, where the ray leaves that
// sphere (spheres that do not contain the origin are skipped), and
// interpolate trilinearly (the azimuth wraps, the poles clamp); opacities are
// per unit of u, so alpha = 1 - exp(-sigma/2).  The foreground renderer takes
// each ray's background colour from here and hands back T_final dL/dC, the
// gradient of that colour (plx_render_opts).
//
// One wave per ray, two samples per lane (2(L-1) = 126 samples for the
// paper's 64 spheres), so even the 5000-ray batches of training keep the
// chip busy: the samples of a ray are independent gathers, and only the
// transmittance couples them, which a wave-wide scan of the optical depths
// provides.  The sample geometry (sphere hit, angles, cell and weights) is
// FP64 in the same operation order as the definition, without contraction,
// so the samples' cells and weights are reproducible; interpolation and
// compositing are FP32 with the optical depth in FP64, as in the foreground.
// The backward pass sums the optical depth (from the same gathers as the
// replay when the ray's samples fit one round of the wave), then walks the
// rounds of samples from the last to the first with suffix scans for the
// depth and the radiance after each sample.
#include <cmath>

#include "plx_internal.hpp"

namespace plx {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr float kY00 = 0.28209479177387814f;
// colour coefficients in record slots 24..26: with the density (slot 28)
// they fill bytes 96..115, one 64-byte line per voxel
constexpr int kSlotR = 24;
// batches of at least this many rays take the lane-per-ray forward
constexpr int64_t kLaneRays = 1 << 17;

struct BgArgs {
    const int32_t *index;
    const float *rec;  // FP32 records
    int L, H, W;
    const float *rays_o;
    const float *rays_d;
    int64_t n_rays;
    float bg[3];
    float *rgb_out;        // fwd
    float *t_out;          // fwd, optional
    const float *grad_rgb; // bwd
    float *grad;           // bwd
    uint8_t *touched;      // bwd
};

// Corner ids and weights of sample k of the ray; false when the sample's
// sphere does not contain the origin.  *cell gets the lower corner's id in
// the grid (for cache keys).
__device__ bool bg_sample(const BgArgs &a, const double o[3], const double d[3], int k, int ids[8],
                          float w[8], int64_t *cell) {
#pragma clang fp contract(off)
    const double u = 0.5 * (double)k;
    const double inv_r = 1.0 - (u + 0.5) / (double)a.L;
    const double r = 1.0 / inv_r;
    const double b = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    const double c = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - r * r;
    if (!(c < 0.0)) return false;
    const double t = -b + sqrt(b * b - c);
    const double p0 = o[0] + t * d[0], p1 = o[1] + t * d[1], p2 = o[2] + t * d[2];
    const double pr = sqrt(p0 * p0 + p1 * p1 + p2 * p2);
    double cz = p2 / pr;
    cz = cz < -1.0 ? -1.0 : (cz > 1.0 ? 1.0 : cz);
    const double theta = acos(cz);
    double phi = atan2(p1, p0);
    if (phi < 0.0) phi += 2.0 * kPi;
    const double gx = phi / (2.0 * kPi) * (double)a.W - 0.5;
    double gy = theta / kPi * (double)a.H - 0.5;
    const double fx0 = floor(gx);
    const double fx = gx - fx0;
    int x0 = (int)fx0;
    x0 = ((x0 % a.W) + a.W) % a.W;
    const int x1 = (x0 + 1) % a.W;
    gy = gy < 0.0 ? 0.0 : (gy > (double)(a.H - 1) ? (double)(a.H - 1) : gy);
    int y0 = (int)floor(gy);
    if (y0 > a.H - 2) y0 = a.H - 2;
    const double fy = gy - y0;
    int l0 = (int)floor(u);
    if (l0 > a.L - 2) l0 = a.L - 2;
    const double fl = u - l0;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
        const int dl = (cc >> 2) & 1, dy = (cc >> 1) & 1, dx = cc & 1;
        const int64_t id = ((int64_t)(l0 + dl) * a.H + (y0 + dy)) * a.W + (dx ? x1 : x0);
        ids[cc] = a.index[id];
        w[cc] = (float)((dl ? fl : 1.0 - fl) * (dy ? fy : 1.0 - fy) * (dx ? fx : 1.0 - fx));
    }
    *cell = ((int64_t)l0 * a.H + y0) * a.W + x0;
    return true;
}

struct BgVal {
    float s, r, g, b;  // pre-activation density and colour coefficients
};

__device__ __forceinline__ void load_ray(const BgArgs &a, int64_t ray, double o[3], double d[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o[i] = (double)a.rays_o[3 * ray + i];
        d[i] = (double)a.rays_d[3 * ray + i];
    }
}

// Wave-wide scans (64 lanes): inclusive prefix sums and exclusive suffix sums.
__device__ __forceinline__ double wave_incl_prefix(double x) {
    const int L = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o);
        if (L >= o) x += y;
    }
    return x;
}
__device__ __forceinline__ float wave_excl_suffix(float x) {
    const int L = threadIdx.x & 63;
    float s = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float y = __shfl_down(s, o);
        if (L + o < 64) s += y;
    }
    return s - x;
}
__device__ __forceinline__ double wave_excl_suffix_d(double x) {
    const int L = threadIdx.x & 63;
    double s = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_down(s, o);
        if (L + o < 64) s += y;
    }
    return s - x;
}
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// One sample of a lane: corners, weights, interpolated values.
struct BgSmp {
    bool ok;
    int ids[8];
    float w[8];
    int64_t cell;
    BgVal v;
};

__device__ __forceinline__ void bg_geom(const BgArgs &a, const double o[3], const double d[3], int k, int n,
                                        BgSmp &s) {
    s.ok = k < n && bg_sample(a, o, d, k, s.ids, s.w, &s.cell);
    if (!s.ok) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            s.ids[c] = -1;
            s.w[c] = 0.0f;
        }
        s.cell = -1;
    }
}

// Colour slots 24..26 and the density (slot 28) of record id.
__device__ __forceinline__ float4 bg_rec(const BgArgs &a, int id) {
    const float *p = a.rec + (int64_t)id * PLX_REC_SLOTS;
    const float4 c = *reinterpret_cast<const float4 *>(p + kSlotR);
    return make_float4(c.x, c.y, c.z, p[PLX_SLOT_SIGMA]);
}

// Samples k (even: on sphere k/2) and k + 1 (halfway to the next sphere)
// with their interpolated values.  A corner's record is read only where its
// weight is non-zero (the even sample's upper corners have weight 0), and
// the odd sample takes its lower corners from the even one when both lie in
// one cell, so a pair reads 8 records where 16 corners are interpolated.
// The sums run over the corners in order, as bg_interp's.
__device__ __forceinline__ void bg_load_pair(const BgArgs &a, const double o[3], const double d[3], int k,
                                             int n, BgSmp &s0, BgSmp &s1) {
    bg_geom(a, o, d, k, n, s0);
    bg_geom(a, o, d, k + 1, n, s1);
    float4 r0[8];
    BgVal v0{0.f, 0.f, 0.f, 0.f}, v1{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const bool need = s0.ids[c] >= 0 && s0.w[c] != 0.0f;
        r0[c] = need ? bg_rec(a, s0.ids[c]) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!(s0.ids[c] >= 0 && s0.w[c] != 0.0f)) continue;
        v0.s += s0.w[c] * r0[c].w;
        v0.r += s0.w[c] * r0[c].x;
        v0.g += s0.w[c] * r0[c].y;
        v0.b += s0.w[c] * r0[c].z;
    }
    const bool same = s0.ok && s1.ok && s0.cell == s1.cell;
    float4 r1[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const bool need = s1.ids[c] >= 0 && s1.w[c] != 0.0f;
        const bool reuse = same && s0.w[c] != 0.0f;
        r1[c] = reuse ? r0[c] : (need ? bg_rec(a, s1.ids[c]) : make_float4(0.f, 0.f, 0.f, 0.f));
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!(s1.ids[c] >= 0 && s1.w[c] != 0.0f)) continue;
        v1.s += s1.w[c] * r1[c].w;
        v1.r += s1.w[c] * r1[c].x;
        v1.g += s1.w[c] * r1[c].y;
        v1.b += s1.w[c] * r1[c].z;
    }
    s0.v = v0;
    s1.v = v1;
}

// One wave per ray; a round covers 128 samples, lane L taking samples
// base + 2L and base + 2L + 1 (the two halves of one layer of cells), so a
// ray's samples are gathered and interpolated in parallel and the
// transmittance comes from a wave-wide scan of their optical depths.
__global__ __launch_bounds__(256) void bg_fwd_kernel(BgArgs a) {
    const int64_t ray = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ray >= a.n_rays) return;
    const int L = threadIdx.x & 63;
    double o[3], d[3];
    load_ray(a, ray, o, d);
    const int n = 2 * (a.L - 1);
    double carry = 0.0;
    float C[3] = {0.f, 0.f, 0.f};
    for (int base = 0; base < n; base += 128) {
        BgSmp s0, s1;
        bg_load_pair(a, o, d, base + 2 * L, n, s0, s1);
        const float sd0 = 0.5f * fmaxf(s0.v.s, 0.0f), sd1 = 0.5f * fmaxf(s1.v.s, 0.0f);
        const double lane_sd = (double)sd0 + (double)sd1;
        const double incl = wave_incl_prefix(lane_sd);
        const double tau0 = carry + (incl - lane_sd);
        const double tau1 = tau0 + (double)sd0;
        const float w0 = expf(-(float)tau0) * (-expm1f(-sd0));
        const float w1 = expf(-(float)tau1) * (-expm1f(-sd1));
        C[0] += w0 * fmaxf(kY00 * s0.v.r, 0.0f) + w1 * fmaxf(kY00 * s1.v.r, 0.0f);
        C[1] += w0 * fmaxf(kY00 * s0.v.g, 0.0f) + w1 * fmaxf(kY00 * s1.v.g, 0.0f);
        C[2] += w0 * fmaxf(kY00 * s0.v.b, 0.0f) + w1 * fmaxf(kY00 * s1.v.b, 0.0f);
        carry += __shfl(incl, 63);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) C[c] = wave_sum(C[c]);
    if (L == 0) {
        const float T = expf(-(float)carry);
#pragma unroll
        for (int c = 0; c < 3; ++c) a.rgb_out[3 * ray + c] = C[c] + T * a.bg[c];
        if (a.t_out) a.t_out[ray] = T;
    }
}

// Value of lane 4*(L/4) + i for every lane L of a quad (all lanes active).
__device__ __forceinline__ int quad_bcast(int x, int i) {
    switch (i) {
    case 0: return __builtin_amdgcn_mov_dpp(x, 0x00, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_mov_dpp(x, 0x55, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_mov_dpp(x, 0xaa, 0xf, 0xf, false);
    default: return __builtin_amdgcn_mov_dpp(x, 0xff, 0xf, 0xf, false);
    }
}
__device__ __forceinline__ float quad_bcast(float x, int i) {
    return __builtin_bit_cast(float, quad_bcast(__builtin_bit_cast(int, x), i));
}

// Adds the gradients acc of corners ids (skipped where !on) to their FP32
// records.  The four values of a voxel (colour slots 24..26 and density slot
// 28, one 64-byte line) are sent by the four lanes of a quad in one
// instruction, one entry of each quad per instruction, so they reach memory
// as one request rather than four.  Called by the whole wave.
__device__ __forceinline__ void bg_flush(const BgArgs &a, const int ids[8], const BgVal acc[8], bool on) {
    const int j = (int)(threadIdx.x & 3);
    const int slot = j < 3 ? kSlotR + j : PLX_SLOT_SIGMA;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int id = on ? ids[c] : -1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idi = quad_bcast(id, i);
            const float t0 = quad_bcast(acc[c].r, i), t1 = quad_bcast(acc[c].g, i);
            const float t2 = quad_bcast(acc[c].b, i), t3 = quad_bcast(acc[c].s, i);
            const float v = j == 0 ? t0 : (j == 1 ? t1 : (j == 2 ? t2 : t3));
            if (idi >= 0 && v != 0.0f) unsafeAtomicAdd(a.grad + (int64_t)idi * PLX_REC_SLOTS + slot, v);
        }
    }
}

__device__ __forceinline__ void bg_mark(const BgArgs &a, const int ids[8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (ids[c] >= 0) a.touched[ids[c]] = 1;
}

// Gradient terms of one sample (dC/dsigma = 1/2 (T_after c - R_after),
// dC/dk_ch = w Y00) spread over its corners.
__device__ __forceinline__ void bg_terms(const BgSmp &s, float w, float T_after, float gR_after,
                                         const float g[3], BgVal acc[8]) {
    const float cr = kY00 * s.v.r, cg = kY00 * s.v.g, cb = kY00 * s.v.b;
    const float gc = g[0] * fmaxf(cr, 0.0f) + g[1] * fmaxf(cg, 0.0f) + g[2] * fmaxf(cb, 0.0f);
    const float dsig = s.v.s > 0.0f ? 0.5f * (T_after * gc - gR_after) : 0.0f;
    const float dr = cr > 0.0f ? w * g[0] * kY00 : 0.0f;
    const float dg = cg > 0.0f ? w * g[1] * kY00 : 0.0f;
    const float db = cb > 0.0f ? w * g[2] * kY00 : 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        acc[c].s += s.w[c] * dsig;
        acc[c].r += s.w[c] * dr;
        acc[c].g += s.w[c] * dg;
        acc[c].b += s.w[c] * db;
    }
}

// One wave per ray: the ray's optical depth by a wave-wide sum, then the
// rounds from the last to the first, each lane's optical depth after its
// samples and the radiance g . R collected after them from wave-wide suffix
// sums; a lane adds its two samples' terms (one set of corners when both lie
// in the same cell) with FP32 atomics.  A lane's second sample lies halfway
// to the next sphere, whose corners at the same angular cell are the lower
// corners of the next lane's first sample: when the cells agree, those four
// corners are handed to the next lane and sent once.
__global__ __launch_bounds__(256) void bg_bwd_kernel(BgArgs a) {
    const int64_t ray = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (ray >= a.n_rays) return;
    const int L = threadIdx.x & 63;
    double o[3], d[3];
    load_ray(a, ray, o, d);
    const int n = 2 * (a.L - 1);
    // With at most 128 samples (64 spheres or fewer) there is one round: its
    // samples give the optical depth as well, so they are gathered once.
    const bool one_round = n <= 128;
    double tau = 0.0;
    if (!one_round) {
        for (int base = 0; base < n; base += 128) {
            BgSmp s0, s1;
            bg_load_pair(a, o, d, base + 2 * L, n, s0, s1);
            tau += (double)(0.5f * fmaxf(s0.v.s, 0.0f)) + (double)(0.5f * fmaxf(s1.v.s, 0.0f));
        }
    }
    const float g[3] = {a.grad_rgb[3 * ray], a.grad_rgb[3 * ray + 1], a.grad_rgb[3 * ray + 2]};
    const float g_bg = g[0] * a.bg[0] + g[1] * a.bg[1] + g[2] * a.bg[2];
    double tau_end = 0.0;  // optical depth after the current round
    float gR_end = 0.0f;
    if (!one_round) {
        tau = wave_sum_d(tau);
        tau_end = tau;
        gR_end = expf(-(float)tau) * g_bg;
    }
    const int last = ((n - 1) / 128) * 128;
    for (int base = last; base >= 0; base -= 128) {
        BgSmp s0, s1;
        bg_load_pair(a, o, d, base + 2 * L, n, s0, s1);
        const float sd0 = 0.5f * fmaxf(s0.v.s, 0.0f), sd1 = 0.5f * fmaxf(s1.v.s, 0.0f);
        const double lane_sd = (double)sd0 + (double)sd1;
        if (one_round) {
            tau_end = wave_sum_d(lane_sd);
            gR_end = expf(-(float)tau_end) * g_bg;
        }
        const double tau_after1 = tau_end - wave_excl_suffix_d(lane_sd);
        const double tau_after0 = fmax(tau_after1 - (double)sd1, 0.0);
        const double tau_before0 = fmax(tau_after0 - (double)sd0, 0.0);
        const float T_after1 = expf(-(float)tau_after1), T_after0 = expf(-(float)tau_after0);
        const float T_before0 = expf(-(float)tau_before0);
        const float w1 = T_after0 * (-expm1f(-sd1)), w0 = T_before0 * (-expm1f(-sd0));
        const float gc1 = g[0] * fmaxf(kY00 * s1.v.r, 0.0f) + g[1] * fmaxf(kY00 * s1.v.g, 0.0f) +
                          g[2] * fmaxf(kY00 * s1.v.b, 0.0f);
        const float gc0 = g[0] * fmaxf(kY00 * s0.v.r, 0.0f) + g[1] * fmaxf(kY00 * s0.v.g, 0.0f) +
                          g[2] * fmaxf(kY00 * s0.v.b, 0.0f);
        const float lane_gR = w0 * gc0 + w1 * gc1;
        const float gR_after1 = gR_end + wave_excl_suffix(lane_gR);
        const float gR_after0 = gR_after1 + w1 * gc1;
        // a1: the second sample's corners; a0: the first's (and the second's
        // when both lie in one cell)
        BgVal a0[8], a1[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) a0[c] = a1[c] = BgVal{0.f, 0.f, 0.f, 0.f};
        if (s1.ok) bg_terms(s1, w1, T_after1, gR_after1, g, a1);
        if (s0.ok) bg_terms(s0, w0, T_after0, gR_after0, g, a0);
        const bool same = s0.ok && s1.ok && s0.cell == s1.cell;
        if (same) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                a0[c].s += a1[c].s;
                a0[c].r += a1[c].r;
                a0[c].g += a1[c].g;
                a0[c].b += a1[c].b;
                a1[c] = BgVal{0.f, 0.f, 0.f, 0.f};
            }
        }
        // hand the second sample's upper corners to the next lane when they
        // are its first sample's lower corners
        const int64_t up_cell = s1.ok ? s1.cell + (int64_t)a.H * a.W : -1;
        const int64_t next_cell = __shfl_down(s0.ok ? s0.cell : (int64_t)-2, 1);
        const bool give = L < 63 && up_cell == next_cell;
        const bool take = __shfl_up(give ? 1 : 0, 1) != 0 && L > 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const BgVal u = same ? a0[4 + c] : a1[4 + c];
            const float rs = __shfl_up(u.s, 1), rr = __shfl_up(u.r, 1);
            const float rg = __shfl_up(u.g, 1), rb = __shfl_up(u.b, 1);
            if (take) {
                a0[c].s += rs;
                a0[c].r += rr;
                a0[c].g += rg;
                a0[c].b += rb;
            }
            if (give) {
                if (same) a0[4 + c] = BgVal{0.f, 0.f, 0.f, 0.f};
                else a1[4 + c] = BgVal{0.f, 0.f, 0.f, 0.f};
            }
        }
        bg_flush(a, s1.ids, a1, s1.ok && !same);
        bg_flush(a, s0.ids, a0, s0.ok);
        if (s1.ok) bg_mark(a, s1.ids);
        if (s0.ok && !same) bg_mark(a, s0.ids);
        tau_end -= __shfl(wave_incl_prefix(lane_sd), 63);
        gR_end += wave_sum(lane_gR);
    }
}

// Lane-per-ray forward for large batches: a lane walks its ray's samples in
// order, so consecutive samples' corner lines stay in its cache; with a
// million rays there are lanes enough to hide the per-sample chain (about
// 20% faster than the wave-per-ray forward there; the wave-per-ray backward
// stays ahead at every size).
__global__ __launch_bounds__(256) void bg_fwd_lane_kernel(BgArgs a) {
    const int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ray >= a.n_rays) return;
    double o[3], d[3];
    load_ray(a, ray, o, d);
    double tau = 0.0;
    float C[3] = {0.f, 0.f, 0.f};
    const int n = 2 * (a.L - 1);
    for (int k = 0; k < n; k += 2) {
        BgSmp sp[2];
        bg_load_pair(a, o, d, k, n, sp[0], sp[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (!sp[h].ok) continue;
            const BgVal v = sp[h].v;
            const float sd = 0.5f * fmaxf(v.s, 0.0f);
            const float wk = expf(-(float)tau) * (-expm1f(-sd));
            C[0] += wk * fmaxf(kY00 * v.r, 0.0f);
            C[1] += wk * fmaxf(kY00 * v.g, 0.0f);
            C[2] += wk * fmaxf(kY00 * v.b, 0.0f);
            tau += (double)sd;
        }
    }
    const float T = expf(-(float)tau);
#pragma unroll
    for (int c = 0; c < 3; ++c) a.rgb_out[3 * ray + c] = C[c] + T * a.bg[c];
    if (a.t_out) a.t_out[ray] = T;
}

int bg_args(const plx_grid *grid, const float *rays_o, const float *rays_d, int64_t n_rays,
            const float background[3], BgArgs &a, const char *fn) {
    int rc = validate_grid(grid, false, fn);
    if (rc) return rc;
    if (grid->sh_dtype != PLX_F32) return fail(PLX_EINVAL, "%s: background records must be FP32", fn);
    if (n_rays < 0 || n_rays > ((int64_t)1 << 34)) return fail(PLX_EINVAL, "%s: bad n_rays", fn);
    if (n_rays > 0 && (!rays_o || !rays_d)) return fail(PLX_EINVAL, "%s: rays are NULL", fn);
    if (!background) return fail(PLX_EINVAL, "%s: background is NULL", fn);
    a = BgArgs{};
    a.index = grid->index;
    a.rec = static_cast<const float *>(grid->data);
    a.L = grid->reso[0];
    a.H = grid->reso[1];
    a.W = grid->reso[2];
    a.rays_o = rays_o;
    a.rays_d = rays_d;
    a.n_rays = n_rays;
    for (int i = 0; i < 3; ++i) a.bg[i] = background[i];
    return PLX_OK;
}

}  // namespace
}  // namespace plx

using namespace plx;

extern "C" {

int plx_bg_render_fwd(const plx_grid *bg_grid, const float *rays_o, const float *rays_d,
                      int64_t n_rays, const float background[3], float *rgb_out, float *t_out,
                      plx_stream stream) {
    const char *fn = "plx_bg_render_fwd";
    BgArgs a;
    int rc = bg_args(bg_grid, rays_o, rays_d, n_rays, background, a, fn);
    if (rc) return rc;
    if (n_rays == 0) return PLX_OK;
    if (!rgb_out) return fail(PLX_EINVAL, "%s: rgb_out is NULL", fn);
    a.rgb_out = rgb_out;
    a.t_out = t_out;
    if (n_rays >= kLaneRays)
        bg_fwd_lane_kernel<<<(unsigned)((n_rays + 255) / 256), 256, 0, as_stream(stream)>>>(a);
    else
        bg_fwd_kernel<<<(unsigned)((n_rays + 3) / 4), 256, 0, as_stream(stream)>>>(a);
    return check_launch(fn);
}

int plx_bg_render_bwd(const plx_grid *bg_grid, const float *rays_o, const float *rays_d,
                      int64_t n_rays, const float background[3], const float *grad_rgb, float *grad,
                      uint8_t *touched, plx_stream stream) {
    const char *fn = "plx_bg_render_bwd";
    BgArgs a;
    int rc = bg_args(bg_grid, rays_o, rays_d, n_rays, background, a, fn);
    if (rc) return rc;
    if (n_rays == 0) return PLX_OK;
    if (!grad_rgb || (bg_grid->n_vox > 0 && (!grad || !touched)))
        return fail(PLX_EINVAL, "%s: NULL grad_rgb/grad/touched", fn);
    a.grad_rgb = grad_rgb;
    a.grad = grad;
    a.touched = touched;
    bg_bwd_kernel<<<(unsigned)((n_rays + 3) / 4), 256, 0, as_stream(stream)>>>(a);
    return check_launch(fn);
}

}  // extern "C"
