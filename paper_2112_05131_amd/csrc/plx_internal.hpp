// plx_internal.hpp -- shared host/device helpers of the gfx950 Plenoxels
// library: error state, launch helpers, the FP32 ray/sample recipe, the SH
// basis and voxel-record access.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/plenoxel.h"

namespace plx {

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);
// Returns PLX_OK, or PLX_EDEVICE (with message) if the last launch failed.
int check_launch(const char *what);

#define PLX_CHECK_HIP(expr, what)                                              \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::plx::fail(PLX_EDEVICE, "%s: %s", (what), hipGetErrorString(e_)); \
    } while (0)

inline hipStream_t as_stream(plx_stream s) { return reinterpret_cast<hipStream_t>(s); }

// Number of set bits among the first n_bits bits of a device bitmap
// (synchronising; ws: caller workspace of PLX_COUNT_WORKSPACE_BYTES).
int count_set_bits(const uint32_t *words, int64_t n_bits, void *ws, int64_t *count_out,
                   hipStream_t s, const char *fn);

// Validates a grid descriptor for kernels; need_occ for the render calls.
int validate_grid(const plx_grid *g, bool need_occ, const char *fn);

inline int64_t n_cells(const int32_t r[3]) { return (int64_t)r[0] * r[1] * r[2]; }

// Bricks of PLX_BRICK^3 cells over the cell lattice 0..N-2 per axis.
inline int bricks_along(int n) { return (n - 1 + PLX_BRICK - 1) / PLX_BRICK; }
inline int64_t n_bricks(const int32_t r[3]) {
    return (int64_t)bricks_along(r[0]) * bricks_along(r[1]) * bricks_along(r[2]);
}
// Cell bitmap: 512 bits (16 words) per brick, bricks in storage order.
inline int64_t occ_words(const int32_t r[3]) {
    return n_bricks(r) * (PLX_BRICK * PLX_BRICK * PLX_BRICK / 32);
}
inline int64_t occ_brick_offset(const int32_t r[3]) { return (occ_words(r) * 4 + 255) / 256 * 256; }

// -------------------------------------------------------- kernel-side grid
struct GridDev {
    int nx, ny, nz;
    int bx, by, bz;  // bricks per axis
    float scale[3], offset[3];
    float step;
    const int32_t *index;
    const void *data;
    const uint32_t *occ;     // cell bitmap
    const uint8_t *bdist;    // brick distances
    int64_t n_vox;
};

inline GridDev to_dev(const plx_grid *g) {
    GridDev d;
    d.nx = g->reso[0];
    d.ny = g->reso[1];
    d.nz = g->reso[2];
    d.bx = bricks_along(d.nx);
    d.by = bricks_along(d.ny);
    d.bz = bricks_along(d.nz);
    for (int a = 0; a < 3; ++a) {
        d.scale[a] = g->scale[a];
        d.offset[a] = g->offset[a];
    }
    d.step = g->step;
    d.index = g->index;
    d.data = g->data;
    d.occ = g->occ;
    d.bdist = g->occ ? reinterpret_cast<const uint8_t *>(g->occ) + occ_brick_offset(g->reso)
                     : nullptr;
    d.n_vox = g->n_vox;
    return d;
}

// Blocks are dispatched round-robin over the 8 XCDs of the chip; this maps a
// hardware block id to a logical one so that each XCD works on one
// contiguous range of logical blocks (its L2 then sees neighbouring work).
// nb8 must be a multiple of 8; logical ids >= the real count are idle.
__device__ inline int xcd_logical_block(int b, int nb8) {
    return (b & 7) * (nb8 >> 3) + (b >> 3);
}
inline int round_up8(int64_t n) { return (int)((n + 7) / 8 * 8); }

// ------------------------------------------------------ FP32 sample recipe
// The discrete decisions (hit, sample count, lower-corner cell) use single
// rounded FP32 operations in a fixed order; contraction into FMAs is off in
// these functions so the results are reproducible bit for bit.
struct RayGeom {
    float og[3], dg[3];
    float t_near, t_far;
};

// Upper bound on samples per ray (FP32 sample parameters stay exact far
// below it; grids up to 2^12 per axis need fewer than 2^14).
constexpr int kMaxSamples = 1 << 22;

// Slab test against the lattice hull [0, N-1]^3.  Returns the sample count
// (0 on a miss).  t_k = t_near + k*step for k < n are exactly the samples
// with t_k < t_far.
__device__ inline int ray_setup(const GridDev &g, const float o[3], const float d[3],
                                RayGeom &r) {
#pragma clang fp contract(off)
    const int reso[3] = {g.nx, g.ny, g.nz};
    float t_near = 0.0f, t_far = __builtin_inff();
    bool hit = true;
    for (int a = 0; a < 3; ++a) {
        float og = o[a] * g.scale[a];
        og = og + g.offset[a];
        float dg = d[a] * g.scale[a];
        float top = (float)(reso[a] - 1);
        r.og[a] = og;
        r.dg[a] = dg;
        if (dg == 0.0f) {
            if (og < 0.0f || og > top) hit = false;
            continue;
        }
        float t0 = (-og) / dg;
        float t1 = (top - og) / dg;
        float tlo = t0 < t1 ? t0 : t1;
        float thi = t0 < t1 ? t1 : t0;
        if (tlo > t_near) t_near = tlo;
        if (thi < t_far) t_far = thi;
    }
    r.t_near = t_near;
    r.t_far = t_far;
    if (!hit || !(t_near < t_far) || !(t_far < __builtin_inff())) return 0;
    // count k with t_near + k*step < t_far, starting from the real quotient
    // (the quotient is within a few units of the count; the adjustment loops
    // are bounded so that no input can keep a wave spinning)
    float span = (t_far - t_near) / g.step;
    if (!(span < (float)kMaxSamples)) span = (float)kMaxSamples;
    int n = (int)ceilf(span);
    if (n < 0) n = 0;
    for (int it = 0; it < 64 && n > 0; ++it) {
        float kk = (float)(n - 1) * g.step;
        if (t_near + kk < t_far) break;
        --n;
    }
    for (int it = 0; it < 64 && n < kMaxSamples; ++it) {
        float kk = (float)n * g.step;
        if (!(t_near + kk < t_far)) break;
        ++n;
    }
    return n;
}

struct Sample {
    int cell[3];   // lower corner
    float f[3];    // position inside the cell, [0, 1]
    float delta;   // interval length
};

__device__ inline Sample sample_at(const GridDev &g, const RayGeom &r, int k) {
#pragma clang fp contract(off)
    Sample s;
    const int reso[3] = {g.nx, g.ny, g.nz};
    float kk = (float)k * g.step;
    float t = r.t_near + kk;
    for (int a = 0; a < 3; ++a) {
        float p = t * r.dg[a];
        float gg = r.og[a] + p;
        int i0 = (int)floorf(gg);
        i0 = i0 < 0 ? 0 : i0;
        i0 = i0 > reso[a] - 2 ? reso[a] - 2 : i0;
        float f = gg - (float)i0;
        f = f < 0.0f ? 0.0f : f;
        f = f > 1.0f ? 1.0f : f;
        s.cell[a] = i0;
        s.f[a] = f;
    }
    float rest = r.t_far - t;
    s.delta = rest < g.step ? rest : g.step;
    return s;
}

__device__ inline int64_t cell_id(const GridDev &g, const int c[3]) {
    return ((int64_t)c[0] * g.ny + c[1]) * (int64_t)g.nz + c[2];
}

// Occupancy bit of the cell with lower corner c: brick (c/8) holds 512 bits,
// cell (i,j,k) of a brick at bit (i%8)*64 + (j%8)*8 + k%8, so the cells a ray
// crosses inside one brick share one 64-byte line.
__device__ inline bool cell_occupied(const GridDev &g, const int c[3]) {
    const int64_t b = ((int64_t)(c[0] >> 3) * g.by + (c[1] >> 3)) * g.bz + (c[2] >> 3);
    const int bit = ((c[0] & 7) << 6) | ((c[1] & 7) << 3) | (c[2] & 7);
    return (g.occ[b * 16 + (bit >> 5)] >> (bit & 31)) & 1u;
}

// ----------------------------------------------------------- SH basis
// Real orthonormal degree-2 SH (Condon-Shortley phase) at direction d, order
// (0,0),(1,-1),(1,0),(1,1),(2,-2),(2,-1),(2,0),(2,1),(2,2).  Evaluated once
// per ray in FP64 and rounded once: 3z^2 - 1 and x^2 - y^2 cancel near their
// zeros, where an FP32 evaluation would lose most of its digits.
__device__ inline float sh_basis_at(int l, float xf, float yf, float zf) {
    const double x = xf, y = yf, z = zf;
    const double k0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
    const double k1 = 0.48860251190291992;   // sqrt(3 / (4 pi))
    const double k2 = 1.09254843059207907;   // sqrt(15 / (4 pi))
    const double k20 = 0.31539156525252005;  // sqrt(5 / (16 pi))
    const double k22 = 0.54627421529603959;  // sqrt(15 / (16 pi))
    double v;
    switch (l) {
    case 0: v = k0; break;
    case 1: v = -k1 * y; break;
    case 2: v = k1 * z; break;
    case 3: v = -k1 * x; break;
    case 4: v = k2 * x * y; break;
    case 5: v = -k2 * y * z; break;
    case 6: v = k20 * (3.0 * z * z - 1.0); break;
    case 7: v = -k2 * x * z; break;
    default: v = k22 * (x * x - y * y); break;
    }
    return (float)v;
}

// ----------------------------------------------------------- records
constexpr int kRecF32Bytes = 128;
constexpr int kRec16Bytes = 64;

template <int DT> struct Rec;

// Record access in two steps so that a caller can issue all its loads before
// converting any of them: raw() loads lane L's chunk (slots 4L..4L+3),
// cvt() turns it into four floats without branches.
template <> struct Rec<PLX_F32> {
    static constexpr int bytes = kRecF32Bytes;
    using Raw = float4;
    __device__ static inline Raw raw(const void *data, int64_t id, int L) {
        const float4 *p = reinterpret_cast<const float4 *>(
            static_cast<const char *>(data) + id * (int64_t)kRecF32Bytes);
        return p[L];
    }
    __device__ static inline Raw zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static inline float4 cvt(Raw r, int) { return r; }
    __device__ static inline float4 load4(const void *data, int64_t id, int L) {
        return raw(data, id, L);
    }
};

__device__ inline float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ inline float f16_to_f32(uint32_t h) {
    return __half2float(__ushort_as_half((unsigned short)h));
}

template <int DT> struct Rec16 {
    static constexpr int bytes = kRec16Bytes;
    using Raw = uint2;
    __device__ static inline float h2f(uint32_t h) {
        return DT == PLX_BF16 ? bf16_to_f32(h) : f16_to_f32(h);
    }
    __device__ static inline Raw raw(const void *data, int64_t id, int L) {
        const uint2 *p = reinterpret_cast<const uint2 *>(
            static_cast<const char *>(data) + id * (int64_t)kRec16Bytes);
        return p[L];
    }
    __device__ static inline Raw zero() { return make_uint2(0u, 0u); }
    // slots 4L..4L+3; lane 7's chunk holds sigma (FP32) in its first word
    __device__ static inline float4 cvt(Raw w, int L) {
        const bool sig = L == 7;
        float4 v;
        v.x = sig ? __uint_as_float(w.x) : h2f(w.x & 0xffffu);
        v.y = sig ? 0.0f : h2f(w.x >> 16);
        v.z = sig ? 0.0f : h2f(w.y & 0xffffu);
        v.w = sig ? 0.0f : h2f(w.y >> 16);
        return v;
    }
    __device__ static inline float4 load4(const void *data, int64_t id, int L) {
        return cvt(raw(data, id, L), L);
    }
};
template <> struct Rec<PLX_BF16> : Rec16<PLX_BF16> {};
template <> struct Rec<PLX_F16> : Rec16<PLX_F16> {};

// Density of record id (any dtype).
template <int DT> __device__ inline float rec_sigma(const void *data, int64_t id) {
    const char *p = static_cast<const char *>(data) + id * (int64_t)Rec<DT>::bytes;
    return DT == PLX_F32 ? reinterpret_cast<const float *>(p)[PLX_SLOT_SIGMA]
                         : *reinterpret_cast<const float *>(p + 56);
}
// Slot s (< 27 or == 28) of record id as float.
template <int DT> __device__ inline float rec_slot(const void *data, int64_t id, int s) {
    if (s == PLX_SLOT_SIGMA) return rec_sigma<DT>(data, id);
    const char *p = static_cast<const char *>(data) + id * (int64_t)Rec<DT>::bytes;
    if (DT == PLX_F32) return reinterpret_cast<const float *>(p)[s];
    uint32_t h = reinterpret_cast<const unsigned short *>(p)[s];
    return DT == PLX_BF16 ? bf16_to_f32(h) : f16_to_f32(h);
}

// Round to nearest even into 16-bit storage.
__device__ inline uint32_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // NaN stays NaN
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return u >> 16;
}
__device__ inline uint32_t f32_to_f16_rne(float x) {
    return (uint32_t)__half_as_ushort(__float2half_rn(x));
}
template <int DT> __device__ inline uint32_t to16(float x) {
    return DT == PLX_BF16 ? f32_to_bf16_rne(x) : f32_to_f16_rne(x);
}

// Dispatch helper over the three storage types.
#define PLX_DISPATCH_DT(dt, DTV, ...)                                          \
    switch (dt) {                                                              \
    case PLX_F32: { constexpr int DTV = PLX_F32; __VA_ARGS__; } break;         \
    case PLX_BF16: { constexpr int DTV = PLX_BF16; __VA_ARGS__; } break;       \
    case PLX_F16: { constexpr int DTV = PLX_F16; __VA_ARGS__; } break;         \
    default: return fail(PLX_EINVAL, "unknown sh_dtype %d", (int)(dt));         \
    }

}  // namespace plx
