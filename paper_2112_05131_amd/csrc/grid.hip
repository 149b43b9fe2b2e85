// grid.hip -- grid create / pack / occupancy / prune / upsample (Sec. 3.2,
// Sec. 3.4, supplement B.1) for gfx950.
//
// Size-changing operations are stream compactions over the cells in storage
// order: a three-phase scan (per-block flag counts, one-block scan of the
// counts, per-block local scan and write).  Table ids therefore follow
// increasing storage id, as the index-grid definition requires.
#include "plx_internal.hpp"

namespace plx {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive scan of one int per thread over a 256-thread block.
__device__ inline int block_exclusive_scan(int x, int *total) {
    __shared__ int wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) {
        off += (i < w) ? wsum[i] : 0;
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

// ---- predicates over cells
struct MaskPred {
    const uint8_t *mask;
    __device__ bool operator()(int64_t v) const { return mask[v] != 0; }
};

struct ParentPred {  // new cell occupied iff its parent cell is occupied
    const int32_t *old_index;
    int on[3], nn[3];
    __device__ bool operator()(int64_t v) const {
        int k = (int)(v % nn[2]);
        int64_t r = v / nn[2];
        int j = (int)(r % nn[1]);
        int i = (int)(r / nn[1]);
        int pi = (int)(((int64_t)(2 * i + 1) * on[0]) / (2 * (int64_t)nn[0]));
        int pj = (int)(((int64_t)(2 * j + 1) * on[1]) / (2 * (int64_t)nn[1]));
        int pk = (int)(((int64_t)(2 * k + 1) * on[2]) / (2 * (int64_t)nn[2]));
        return old_index[((int64_t)pi * on[1] + pj) * on[2] + pk] >= 0;
    }
};

template <class Pred>
__global__ __launch_bounds__(kScanThreads) void scan_count_kernel(Pred pred, int64_t n,
                                                                  int *counts) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int c = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t v = base + i;
        if (v < n && pred(v)) ++c;
    }
    int tot;
    block_exclusive_scan(c, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// One block: exclusive scan of nb block counts into offsets[0..nb], offsets[nb]
// = total.
__global__ __launch_bounds__(kScanThreads) void scan_offsets_kernel(const int *counts, int64_t nb,
                                                                    int64_t *offsets) {
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        int64_t b = b0 + threadIdx.x;
        int c = b < nb ? counts[b] : 0;
        int tot;
        int ex = block_exclusive_scan(c, &tot);
        int64_t base = carry;
        if (b < nb) offsets[b] = base + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = base + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[nb] = carry;
}

template <class Pred, class Writer>
__global__ __launch_bounds__(kScanThreads) void scan_write_kernel(Pred pred, Writer wr, int64_t n,
                                                                  const int64_t *offsets) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t flags = 0;
    int c = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t v = base + i;
        if (v < n && pred(v)) {
            flags |= 1u << i;
            ++c;
        }
    }
    int tot;
    int64_t rank = offsets[blockIdx.x] + block_exclusive_scan(c, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t v = base + i;
        if (v >= n) break;
        if (flags & (1u << i)) {
            wr.occupied(v, rank);
            ++rank;
        } else {
            wr.empty(v);
        }
    }
}

// Workspace of the grid calls (caller-owned, plx_grid_workspace_bytes): a
// 256-byte block of counters, then one byte per cell (the prune occupancy
// flags), then the per-block counts and offsets of the compaction scan.
struct WsLayout {
    int64_t counters, bytes8, scan, bytes;
};
inline int64_t up256(int64_t x) { return (x + 255) / 256 * 256; }
inline int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }
WsLayout ws_layout(int64_t ncell) {
    WsLayout l;
    l.counters = 0;
    l.bytes8 = 256;
    l.scan = l.bytes8 + up256(ncell);
    const int64_t nb = scan_blocks(ncell);
    l.bytes = l.scan + up256((nb + 1) * 8) + up256(nb * 4);
    return l;
}

int check_ws(const void *ws, int64_t ws_bytes, int64_t need, const char *fn) {
    if (!ws) return fail(PLX_EINVAL, "%s: workspace is NULL", fn);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PLX_EINVAL, "%s: workspace must be 256-byte aligned", fn);
    if (ws_bytes < need)
        return fail(PLX_EINVAL, "%s: workspace of %lld bytes, need %lld", fn, (long long)ws_bytes, (long long)need);
    return PLX_OK;
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0ull;
}

// Clears the workspace's counters (a kernel rather than a memset node, so
// that a captured graph replays it like any other launch).
int zero_counters(void *ws, hipStream_t s, const char *fn) {
    zero_u64_kernel<<<1, 32, 0, s>>>(static_cast<unsigned long long *>(ws), 32);
    return check_launch(fn);
}

template <class Pred, class Writer>
int run_scan(Pred pred, Writer wr, int64_t n, void *ws, hipStream_t s, const char *what) {
    if (n <= 0) return PLX_OK;
    int64_t nb = scan_blocks(n);
    if (nb > 0x7fffffff) return fail(PLX_EINVAL, "%s: too many cells", what);
    const WsLayout l = ws_layout(n);
    int64_t *offsets = reinterpret_cast<int64_t *>(static_cast<char *>(ws) + l.scan);
    int *counts = reinterpret_cast<int *>(static_cast<char *>(ws) + l.scan + up256((nb + 1) * 8));
    int rc;
    scan_count_kernel<<<(unsigned)nb, kScanThreads, 0, s>>>(pred, n, counts);
    if ((rc = check_launch(what))) return rc;
    scan_offsets_kernel<<<1, kScanThreads, 0, s>>>(counts, nb, offsets);
    if ((rc = check_launch(what))) return rc;
    scan_write_kernel<<<(unsigned)nb, kScanThreads, 0, s>>>(pred, wr, n, offsets);
    return check_launch(what);
}

// ---- writers
struct IndexWriter {
    int32_t *out;
    __device__ void occupied(int64_t v, int64_t rank) const { out[v] = (int32_t)rank; }
    __device__ void empty(int64_t v) const { out[v] = -1; }
};

struct PruneWriter {
    int32_t *out;
    const int32_t *old_index;
    const uint4 *old_data;  // records as 16-byte chunks
    uint4 *new_data;
    int chunks;             // 16-byte chunks per record
    __device__ void occupied(int64_t v, int64_t rank) const {
        out[v] = (int32_t)rank;
        int64_t src = (int64_t)old_index[v] * chunks, dst = rank * chunks;
        for (int c = 0; c < chunks; ++c) new_data[dst + c] = old_data[src + c];
    }
    __device__ void empty(int64_t v) const { out[v] = -1; }
};

// ---- small kernels

// Counting kernels run a fixed grid of kCountBlocks x kCountThreads threads
// that stride over the input; each block adds its total to the counter with
// one atomic (one atomic per wave on a single address serialises: 2M of them
// for a 512^3 mask).
constexpr int kCountThreads = 256;
constexpr int64_t kCountBlocks = 2048;

inline unsigned count_blocks(int64_t n) {
    const int64_t b = (n + kCountThreads - 1) / kCountThreads;
    return (unsigned)(b < 1 ? 1 : (b > kCountBlocks ? kCountBlocks : b));
}

__device__ void block_add(unsigned long long v, unsigned long long *out) {
    __shared__ unsigned long long part[kCountThreads / 64];
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kCountThreads / 64; ++w) t += part[w];
        if (t) atomicAdd(out, t);
    }
}

// Adds the block's totals of v0 and v1 to out[0] and out[1].
__device__ void block_add2(unsigned long long v0, unsigned long long v1, unsigned long long *out) {
    __shared__ unsigned long long part[2][kCountThreads / 64];
    for (int o = 32; o >= 1; o >>= 1) {
        v0 += __shfl_xor(v0, o);
        v1 += __shfl_xor(v1, o);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = v0;
        part[1][threadIdx.x >> 6] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t0 = 0, t1 = 0;
        for (int w = 0; w < kCountThreads / 64; ++w) {
            t0 += part[0][w];
            t1 += part[1][w];
        }
        if (t0) atomicAdd(out, t0);
        if (t1) atomicAdd(out + 1, t1);
    }
}

// Number of non-zero bytes of m[0..n).
__global__ __launch_bounds__(kCountThreads) void count_nonzero_kernel(const uint8_t *m, int64_t n,
                                                                      unsigned long long *out) {
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kCountThreads + threadIdx.x; i < n; i += stride)
        c += m[i] != 0;
    block_add(c, out);
}

// Number of set bits among the first nbits bits of w[0..nw).
__global__ __launch_bounds__(kCountThreads) void popcount_kernel(const uint32_t *w, int64_t nw,
                                                                 int64_t nbits,
                                                                 unsigned long long *out) {
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kCountThreads + threadIdx.x; i < nw; i += stride) {
        uint32_t x = w[i];
        const int64_t first = i * 32;
        if (first + 32 > nbits) {
            const int keep = (int)(nbits - first);
            x &= keep >= 32 ? 0xffffffffu : ((1u << keep) - 1u);
        }
        c += __popc(x);
    }
    block_add(c, out);
}

template <int DT>
__global__ void pack_kernel(int64_t n, const float *density, const float *sh, float sigma0,
                            float dc, void *out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 8) return;
    int64_t m = t >> 3;
    int L = (int)(t & 7);
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        int s = 4 * L + e;
        float x = 0.0f;
        if (s < PLX_NSH)
            x = sh ? sh[m * PLX_NSH + s] : ((s % 9) == 0 ? dc : 0.0f);
        else if (s == PLX_SLOT_SIGMA)
            x = density ? density[m] : sigma0;
        v[e] = x;
    }
    if (DT == PLX_F32) {
        reinterpret_cast<float4 *>(static_cast<char *>(out) + m * kRecF32Bytes)[L] =
            make_float4(v[0], v[1], v[2], v[3]);
    } else {
        uint2 w;
        if (L == 7) {
            w.x = __float_as_uint(v[0]);
            w.y = 0u;
        } else {
            w.x = to16<DT>(v[0]) | (to16<DT>(v[1]) << 16);
            w.y = to16<DT>(v[2]) | (to16<DT>(v[3]) << 16);
            if (L == 6) w.y &= 0xffffu;  // slot 27 unused
        }
        reinterpret_cast<uint2 *>(static_cast<char *>(out) + m * kRec16Bytes)[L] = w;
    }
}

template <int DT>
__global__ void unpack_kernel(int64_t n, const void *rec, float *density, float *sh) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 32) return;
    int64_t m = t >> 5;
    int s = (int)(t & 31);
    if (s < PLX_NSH) {
        if (sh) sh[m * PLX_NSH + s] = rec_slot<DT>(rec, m, s);
    } else if (s == PLX_SLOT_SIGMA) {
        if (density) density[m] = rec_sigma<DT>(rec, m);
    }
}

// Cell occupancy bits in brick-major order: thread t is bit t of the bitmap,
// i.e. brick t/512, cell (t%512)/64, (t/8)%8, t%8 inside it; 32-bit words are
// assembled by ballot.  Cells outside the lattice (partial bricks) get 0.
__global__ void occupancy_kernel(GridDev g, int64_t nbits, uint32_t *occ) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bit = false;
    if (t < nbits) {
        const int64_t b = t >> 9;
        const int l = (int)(t & 511);
        const int bk = (int)(b % g.bz);
        const int bj = (int)((b / g.bz) % g.by);
        const int bi = (int)(b / ((int64_t)g.bz * g.by));
        const int i = bi * PLX_BRICK + (l >> 6), j = bj * PLX_BRICK + ((l >> 3) & 7),
                  k = bk * PLX_BRICK + (l & 7);
        if (i < g.nx - 1 && j < g.ny - 1 && k < g.nz - 1) {
            const int64_t sy = g.nz, sx = (int64_t)g.ny * g.nz;
            const int32_t *p = g.index + ((int64_t)i * g.ny + j) * g.nz + k;
            // NULL entries are negative, table ids are not: the cell is empty
            // exactly when the AND of all eight entries is negative
            bit = (p[0] & p[1] & p[sy] & p[sy + 1] & p[sx] & p[sx + 1] & p[sx + sy] &
                   p[sx + sy + 1]) >= 0;
        }
    }
    const unsigned long long m = __ballot(bit);
    const int lane = threadIdx.x & 63;
    const int64_t w = (t - lane) >> 5;  // first word of this wave
    if (lane == 0 && (t - lane) < nbits) occ[w] = (uint32_t)(m & 0xffffffffull);
    if (lane == 32 && (t - lane) + 32 < nbits) occ[w + 1] = (uint32_t)(m >> 32);
}

// Brick seed: 0 when any cell of the brick has its occupancy bit, else far.
__global__ void brick_seed_kernel(GridDev g, uint8_t *bd) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (int64_t)g.bx * g.by * g.bz;
    if (b >= nb) return;
    uint32_t any = 0u;
    for (int w = 0; w < 16; ++w) any |= g.occ[b * 16 + w];
    bd[b] = any ? 0 : 255;
}

// One relaxation pass of the Chebyshev distance over bricks, in place:
// d <- min(d, 1 + min over the 26 neighbours).  Every value stays an upper
// bound of the true distance; `last` clamps to the cap, which turns the
// values of unconverged (far) bricks into lower bounds.
__global__ void brick_dist_pass_kernel(GridDev g, uint8_t *bd, int last) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (int64_t)g.bx * g.by * g.bz;
    if (b >= nb) return;
    const int bk = (int)(b % g.bz);
    const int bj = (int)((b / g.bz) % g.by);
    const int bi = (int)(b / ((int64_t)g.bz * g.by));
    int d = bd[b];
    for (int a = -1; a <= 1; ++a) {
        const int ii = bi + a;
        if (ii < 0 || ii >= g.bx) continue;
        for (int c = -1; c <= 1; ++c) {
            const int jj = bj + c;
            if (jj < 0 || jj >= g.by) continue;
            for (int e = -1; e <= 1; ++e) {
                const int kk = bk + e;
                if (kk < 0 || kk >= g.bz) continue;
                const int nd = bd[((int64_t)ii * g.by + jj) * g.bz + kk] + 1;
                d = nd < d ? nd : d;
            }
        }
    }
    if (last) d = d < PLX_BRICK_DIST_CAP ? d : PLX_BRICK_DIST_CAP;
    bd[b] = (uint8_t)d;
}

template <int DT>
__global__ void prune_occ_kernel(GridDev g, int64_t ncell, float thresh, uint8_t *occ8) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= ncell) return;
    int32_t id = g.index[v];
    occ8[v] = (id >= 0 && rec_sigma<DT>(g.data, id) >= thresh) ? 1 : 0;
}

__global__ void prune_occ_value_kernel(GridDev g, int64_t ncell, const float *value, float thresh,
                                      uint8_t *occ8) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= ncell) return;
    int32_t id = g.index[v];
    occ8[v] = (id >= 0 && value[id] >= thresh) ? 1 : 0;
}

__global__ __launch_bounds__(kCountThreads) void prune_keep_kernel(GridDev g, int64_t ncell,
                                                                   const uint8_t *occ8, uint8_t *keep,
                                                                   unsigned long long *counts) {
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    unsigned long long n_kept = 0, n_nonnull = 0;
    for (int64_t v = (int64_t)blockIdx.x * kCountThreads + threadIdx.x; v < ncell; v += stride) {
        bool nonnull = false, kept = false;
        int k = (int)(v % g.nz);
        int64_t r = v / g.nz;
        int j = (int)(r % g.ny);
        int i = (int)(r / g.ny);
        nonnull = g.index[v] >= 0;
        if (nonnull) {
            for (int a = -1; a <= 1 && !kept; ++a) {
                int ii = i + a;
                if (ii < 0 || ii >= g.nx) continue;
                for (int b = -1; b <= 1 && !kept; ++b) {
                    int jj = j + b;
                    if (jj < 0 || jj >= g.ny) continue;
                    for (int c = -1; c <= 1; ++c) {
                        int kk = k + c;
                        if (kk < 0 || kk >= g.nz) continue;
                        if (occ8[((int64_t)ii * g.ny + jj) * g.nz + kk]) {
                            kept = true;
                            break;
                        }
                    }
                }
            }
        }
        keep[v] = kept ? 1 : 0;
        n_kept += kept;
        n_nonnull += nonnull;
    }
    block_add2(n_kept, n_nonnull, counts);
}

__global__ __launch_bounds__(kCountThreads) void upsample_count_kernel(ParentPred pred, int64_t n,
                                                                       unsigned long long *out) {
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    unsigned long long c = 0;
    for (int64_t v = (int64_t)blockIdx.x * kCountThreads + threadIdx.x; v < n; v += stride)
        c += pred(v) ? 1 : 0;
    block_add(c, out);
}

// Old-grid coordinate of new voxel j (FP64, same operation order as the
// definition): ((j + 0.5) N_old / N_new) - 0.5, clamped to [0, N_old - 1].
__device__ inline void upsample_coord(int j, int n_old, int n_new, int &i0, double &f) {
    double g = ((double)j + 0.5) * (double)n_old / (double)n_new - 0.5;
    if (g < 0.0) g = 0.0;
    if (g > (double)(n_old - 1)) g = (double)(n_old - 1);
    int c = (int)floor(g);
    if (c > n_old - 2) c = n_old - 2;
    if (c < 0) c = 0;
    i0 = c;
    f = g - (double)c;
}

template <int DT>
__global__ void upsample_values_kernel(GridDev go, const int32_t *new_index, int nn0, int nn1,
                                       int nn2, int64_t ncell_new, void *new_data) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= ncell_new) return;
    int32_t nid = new_index[v];
    if (nid < 0) return;
    int k = (int)(v % nn2);
    int64_t r = v / nn2;
    int j = (int)(r % nn1);
    int i = (int)(r / nn1);
    int c0[3];
    double f[3];
    upsample_coord(i, go.nx, nn0, c0[0], f[0]);
    upsample_coord(j, go.ny, nn1, c0[1], f[1]);
    upsample_coord(k, go.nz, nn2, c0[2], f[2]);
    double acc[29];
    for (int s = 0; s < 29; ++s) acc[s] = 0.0;
    for (int c = 0; c < 8; ++c) {
        int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
        double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        int64_t id = go.index[((int64_t)(c0[0] + dx) * go.ny + (c0[1] + dy)) * go.nz + (c0[2] + dz)];
        if (id < 0) continue;
        for (int s = 0; s < PLX_NSH; ++s) acc[s] += w * (double)rec_slot<DT>(go.data, id, s);
        acc[PLX_SLOT_SIGMA] += w * (double)rec_sigma<DT>(go.data, id);
    }
    if (DT == PLX_F32) {
        float *o = reinterpret_cast<float *>(static_cast<char *>(new_data) + (int64_t)nid * kRecF32Bytes);
        for (int s = 0; s < 32; ++s)
            o[s] = (s < PLX_NSH || s == PLX_SLOT_SIGMA) ? (float)acc[s] : 0.0f;
    } else {
        char *o = static_cast<char *>(new_data) + (int64_t)nid * kRec16Bytes;
        unsigned short *h = reinterpret_cast<unsigned short *>(o);
        for (int s = 0; s < 28; ++s) h[s] = s < PLX_NSH ? (unsigned short)to16<DT>((float)acc[s]) : 0;
        float *sg = reinterpret_cast<float *>(o + 56);
        sg[0] = (float)acc[PLX_SLOT_SIGMA];
        sg[1] = 0.0f;
    }
}

template <int DS, int DD>
__global__ void convert_kernel(int64_t n, const void *src, void *dst) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 8) return;
    int64_t m = t >> 3;
    int L = (int)(t & 7);
    float4 x = Rec<DS>::load4(src, m, L);
    float v[4] = {x.x, x.y, x.z, x.w};
    if (DD == PLX_F32) {
        reinterpret_cast<float4 *>(static_cast<char *>(dst) + m * kRecF32Bytes)[L] =
            make_float4(v[0], v[1], v[2], v[3]);
    } else {
        uint2 w;
        if (L == 7) {
            w.x = __float_as_uint(v[0]);
            w.y = 0u;
        } else {
            w.x = to16<DD>(v[0]) | (to16<DD>(v[1]) << 16);
            w.y = to16<DD>(v[2]) | (to16<DD>(v[3]) << 16);
            if (L == 6) w.y &= 0xffffu;
        }
        reinterpret_cast<uint2 *>(static_cast<char *>(dst) + m * kRec16Bytes)[L] = w;
    }
}

int sync_read_u64(const unsigned long long *dev, int n, int64_t *host, hipStream_t s,
                  const char *what) {
    unsigned long long tmp[4] = {0, 0, 0, 0};
    PLX_CHECK_HIP(hipMemcpyAsync(tmp, dev, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
                  what);
    PLX_CHECK_HIP(hipStreamSynchronize(s), what);
    for (int i = 0; i < n; ++i) host[i] = (int64_t)tmp[i];
    return PLX_OK;
}

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }


// Shared by both prune counts: occupied = non-NULL with density (value ==
// NULL) or value[id] at least thresh; kept = non-NULL with an occupied voxel
// in its 3x3x3 neighbourhood.
int prune_count(const plx_grid *grid, const float *value, float thresh, uint8_t *keep_out, void *ws,
                int64_t ws_bytes, int64_t *n_kept, int64_t *n_pruned, plx_stream stream,
                const char *fn) {
    int rc = validate_grid(grid, false, fn);
    if (rc) return rc;
    if (!keep_out || !n_kept || !n_pruned) return fail(PLX_EINVAL, "%s: NULL argument", fn);
    hipStream_t s = as_stream(stream);
    int64_t ncell = n_cells(grid->reso);
    const WsLayout l = ws_layout(ncell);
    if ((rc = check_ws(ws, ws_bytes, l.bytes, fn))) return rc;
    auto *counts = static_cast<unsigned long long *>(ws);
    uint8_t *occ8 = static_cast<uint8_t *>(ws) + l.bytes8;
    if ((rc = zero_counters(ws, s, fn))) return rc;
    GridDev g = to_dev(grid);
    unsigned nb = blocks_for(ncell, 256);
    if (value) {
        prune_occ_value_kernel<<<nb, 256, 0, s>>>(g, ncell, value, thresh, occ8);
    } else {
        PLX_DISPATCH_DT(grid->sh_dtype, DT,
                        prune_occ_kernel<DT><<<nb, 256, 0, s>>>(g, ncell, thresh, occ8));
    }
    if ((rc = check_launch(fn))) return rc;
    prune_keep_kernel<<<count_blocks(ncell), kCountThreads, 0, s>>>(g, ncell, occ8, keep_out, counts);
    if ((rc = check_launch(fn))) return rc;
    int64_t h[2];
    if ((rc = sync_read_u64(counts, 2, h, s, fn))) return rc;
    *n_kept = h[0];
    *n_pruned = h[1] - h[0];
    return PLX_OK;
}

}  // namespace
}  // namespace plx

using namespace plx;

extern "C" {

int64_t plx_grid_workspace_bytes(const int32_t reso[3]) {
    if (!reso || reso[0] < 2 || reso[1] < 2 || reso[2] < 2) return 0;
    return ws_layout(n_cells(reso)).bytes;
}

int plx_mask_count(const uint8_t *mask, int64_t n, void *ws, int64_t ws_bytes, int64_t *count_out,
                   plx_stream stream) {
    if (!count_out) return fail(PLX_EINVAL, "plx_mask_count: count_out is NULL");
    if (n < 0) return fail(PLX_EINVAL, "plx_mask_count: n < 0");
    int rc = check_ws(ws, ws_bytes, PLX_COUNT_WORKSPACE_BYTES, "plx_mask_count");
    if (rc) return rc;
    if (n == 0) {
        *count_out = 0;
        return PLX_OK;
    }
    if (!mask) return fail(PLX_EINVAL, "plx_mask_count: mask is NULL");
    hipStream_t s = as_stream(stream);
    auto *cnt = static_cast<unsigned long long *>(ws);
    if ((rc = zero_counters(ws, s, "plx_mask_count"))) return rc;
    count_nonzero_kernel<<<count_blocks(n), kCountThreads, 0, s>>>(mask, n, cnt);
    if ((rc = check_launch("plx_mask_count"))) return rc;
    return sync_read_u64(cnt, 1, count_out, s, "plx_mask_count");
}

int plx_grid_create(const uint8_t *mask, const int32_t reso[3], int32_t *index_out, void *ws,
                    int64_t ws_bytes, plx_stream stream) {
    if (!mask || !reso || !index_out) return fail(PLX_EINVAL, "plx_grid_create: NULL argument");
    for (int a = 0; a < 3; ++a)
        if (reso[a] < 2) return fail(PLX_EINVAL, "plx_grid_create: reso[%d] < 2", a);
    int64_t n = n_cells(reso);
    int rc = check_ws(ws, ws_bytes, ws_layout(n).bytes, "plx_grid_create");
    if (rc) return rc;
    return run_scan(MaskPred{mask}, IndexWriter{index_out}, n, ws, as_stream(stream), "plx_grid_create");
}

int plx_records_pack(int32_t sh_dtype, int64_t n, const float *density, const float *sh,
                     float sigma0, float dc, void *out, plx_stream stream) {
    if (n < 0) return fail(PLX_EINVAL, "plx_records_pack: n < 0");
    if (n == 0) return PLX_OK;
    if (!out) return fail(PLX_EINVAL, "plx_records_pack: out is NULL");
    hipStream_t s = as_stream(stream);
    PLX_DISPATCH_DT(sh_dtype, DT,
                    pack_kernel<DT><<<blocks_for(n * 8, 256), 256, 0, s>>>(n, density, sh, sigma0,
                                                                           dc, out));
    return check_launch("plx_records_pack");
}

int plx_records_unpack(int32_t sh_dtype, int64_t n, const void *records, float *density,
                       float *sh, plx_stream stream) {
    if (n < 0) return fail(PLX_EINVAL, "plx_records_unpack: n < 0");
    if (n == 0) return PLX_OK;
    if (!records) return fail(PLX_EINVAL, "plx_records_unpack: records is NULL");
    hipStream_t s = as_stream(stream);
    PLX_DISPATCH_DT(sh_dtype, DT,
                    unpack_kernel<DT><<<blocks_for(n * 32, 256), 256, 0, s>>>(n, records, density, sh));
    return check_launch("plx_records_unpack");
}

int plx_records_convert(int32_t src_dtype, const void *src, int32_t dst_dtype, void *dst,
                        int64_t n, plx_stream stream) {
    if (n < 0) return fail(PLX_EINVAL, "plx_records_convert: n < 0");
    if (n == 0) return PLX_OK;
    if (!src || !dst) return fail(PLX_EINVAL, "plx_records_convert: NULL argument");
    hipStream_t s = as_stream(stream);
    unsigned nb = blocks_for(n * 8, 256);
    PLX_DISPATCH_DT(src_dtype, DS,
                    PLX_DISPATCH_DT(dst_dtype, DD,
                                    convert_kernel<DS, DD><<<nb, 256, 0, s>>>(n, src, dst)));
    return check_launch("plx_records_convert");
}

int plx_grid_build_occupancy(const plx_grid *grid, uint32_t *occ_out, plx_stream stream) {
    int rc = validate_grid(grid, false, "plx_grid_build_occupancy");
    if (rc) return rc;
    if (!occ_out) return fail(PLX_EINVAL, "plx_grid_build_occupancy: occ_out is NULL");
    hipStream_t s = as_stream(stream);
    // bits are whole bricks of 512, so whole waves: every word is written by
    // the wave that owns it
    const int64_t nbits = occ_words(grid->reso) * 32;
    plx_grid gd = *grid;
    gd.occ = occ_out;
    GridDev g = to_dev(&gd);
    occupancy_kernel<<<blocks_for(nbits, 256), 256, 0, s>>>(g, nbits, occ_out);
    if ((rc = check_launch("plx_grid_build_occupancy"))) return rc;
    uint8_t *bd = reinterpret_cast<uint8_t *>(occ_out) + occ_brick_offset(grid->reso);
    const int64_t nb = n_bricks(grid->reso);
    brick_seed_kernel<<<blocks_for(nb, 256), 256, 0, s>>>(g, bd);
    if ((rc = check_launch("plx_grid_build_occupancy"))) return rc;
    for (int p = 0; p < PLX_BRICK_DIST_CAP; ++p) {
        brick_dist_pass_kernel<<<blocks_for(nb, 256), 256, 0, s>>>(g, bd, p == PLX_BRICK_DIST_CAP - 1);
        if ((rc = check_launch("plx_grid_build_occupancy"))) return rc;
    }
    return PLX_OK;
}

int plx_grid_prune_count(const plx_grid *grid, float sigma_thresh, uint8_t *keep_out, void *ws,
                         int64_t ws_bytes, int64_t *n_kept, int64_t *n_pruned, plx_stream stream) {
    return plx::prune_count(grid, nullptr, sigma_thresh, keep_out, ws, ws_bytes, n_kept, n_pruned,
                            stream, "plx_grid_prune_count");
}

int plx_grid_prune_weight_count(const plx_grid *grid, const float *wmax, float w_thresh,
                                uint8_t *keep_out, void *ws, int64_t ws_bytes, int64_t *n_kept,
                                int64_t *n_pruned, plx_stream stream) {
    if (!wmax) return plx::fail(PLX_EINVAL, "plx_grid_prune_weight_count: wmax is NULL");
    return plx::prune_count(grid, wmax, w_thresh, keep_out, ws, ws_bytes, n_kept, n_pruned, stream,
                            "plx_grid_prune_weight_count");
}

int plx_grid_prune_apply(const plx_grid *grid, const uint8_t *keep, plx_grid *out, void *ws,
                         int64_t ws_bytes, plx_stream stream) {
    int rc = validate_grid(grid, false, "plx_grid_prune_apply");
    if (rc) return rc;
    if (!keep || !out || !out->index) return fail(PLX_EINVAL, "plx_grid_prune_apply: NULL argument");
    for (int a = 0; a < 3; ++a)
        if (out->reso[a] != grid->reso[a])
            return fail(PLX_EINVAL, "plx_grid_prune_apply: out->reso differs from grid->reso");
    if (out->sh_dtype != grid->sh_dtype)
        return fail(PLX_EINVAL, "plx_grid_prune_apply: out->sh_dtype differs");
    if (out->n_vox > 0 && !out->data) return fail(PLX_EINVAL, "plx_grid_prune_apply: out->data is NULL");
    int chunks = (int)(plx_record_bytes(grid->sh_dtype) / 16);
    PruneWriter w{const_cast<int32_t *>(out->index), grid->index, static_cast<const uint4 *>(grid->data),
                  static_cast<uint4 *>(out->data), chunks};
    if ((rc = check_ws(ws, ws_bytes, ws_layout(n_cells(grid->reso)).bytes, "plx_grid_prune_apply"))) return rc;
    return run_scan(MaskPred{keep}, w, n_cells(grid->reso), ws, as_stream(stream), "plx_grid_prune_apply");
}

int plx_grid_upsample_count(const plx_grid *grid, const int32_t new_reso[3], void *ws,
                            int64_t ws_bytes, int64_t *n_out, plx_stream stream) {
    int rc = validate_grid(grid, false, "plx_grid_upsample_count");
    if (rc) return rc;
    if (!new_reso || !n_out) return fail(PLX_EINVAL, "plx_grid_upsample_count: NULL argument");
    for (int a = 0; a < 3; ++a)
        if (new_reso[a] < 2) return fail(PLX_EINVAL, "plx_grid_upsample_count: new_reso[%d] < 2", a);
    hipStream_t s = as_stream(stream);
    ParentPred pred{grid->index, {grid->reso[0], grid->reso[1], grid->reso[2]},
                    {new_reso[0], new_reso[1], new_reso[2]}};
    int64_t n = n_cells(new_reso);
    if ((rc = check_ws(ws, ws_bytes, PLX_COUNT_WORKSPACE_BYTES, "plx_grid_upsample_count"))) return rc;
    auto *cnt = static_cast<unsigned long long *>(ws);
    if ((rc = zero_counters(ws, s, "plx_grid_upsample_count"))) return rc;
    upsample_count_kernel<<<count_blocks(n), kCountThreads, 0, s>>>(pred, n, cnt);
    if ((rc = check_launch("plx_grid_upsample_count"))) return rc;
    return sync_read_u64(cnt, 1, n_out, s, "plx_grid_upsample_count");
}

int plx_grid_upsample_apply(const plx_grid *grid, plx_grid *out, void *ws, int64_t ws_bytes,
                            plx_stream stream) {
    int rc = validate_grid(grid, false, "plx_grid_upsample_apply");
    if (rc) return rc;
    if (!out || !out->index) return fail(PLX_EINVAL, "plx_grid_upsample_apply: NULL argument");
    for (int a = 0; a < 3; ++a)
        if (out->reso[a] < 2) return fail(PLX_EINVAL, "plx_grid_upsample_apply: out->reso[%d] < 2", a);
    if (out->sh_dtype != grid->sh_dtype)
        return fail(PLX_EINVAL, "plx_grid_upsample_apply: out->sh_dtype differs from grid->sh_dtype");
    if (out->n_vox > 0 && !out->data) return fail(PLX_EINVAL, "plx_grid_upsample_apply: out->data is NULL");
    hipStream_t s = as_stream(stream);
    ParentPred pred{grid->index, {grid->reso[0], grid->reso[1], grid->reso[2]},
                    {out->reso[0], out->reso[1], out->reso[2]}};
    int64_t n = n_cells(out->reso);
    if ((rc = check_ws(ws, ws_bytes, ws_layout(n).bytes, "plx_grid_upsample_apply"))) return rc;
    if ((rc = run_scan(pred, IndexWriter{const_cast<int32_t *>(out->index)}, n, ws, s,
                       "plx_grid_upsample_apply")))
        return rc;
    GridDev g = to_dev(grid);
    PLX_DISPATCH_DT(grid->sh_dtype, DT,
                    upsample_values_kernel<DT><<<blocks_for(n, 256), 256, 0, s>>>(
                        g, out->index, out->reso[0], out->reso[1], out->reso[2], n, out->data));
    return check_launch("plx_grid_upsample_apply");
}

int plx_touched_count(const uint8_t *touched, int64_t n_vox, void *ws, int64_t ws_bytes,
                      int64_t *count_out, plx_stream stream) {
    if (!count_out) return fail(PLX_EINVAL, "plx_touched_count: count_out is NULL");
    if (n_vox < 0) return fail(PLX_EINVAL, "plx_touched_count: n_vox < 0");
    int rc = check_ws(ws, ws_bytes, PLX_COUNT_WORKSPACE_BYTES, "plx_touched_count");
    if (rc) return rc;
    if (n_vox == 0) {
        *count_out = 0;
        return PLX_OK;
    }
    if (!touched) return fail(PLX_EINVAL, "plx_touched_count: touched is NULL");
    hipStream_t s = as_stream(stream);
    auto *cnt = static_cast<unsigned long long *>(ws);
    if ((rc = zero_counters(ws, s, "plx_touched_count"))) return rc;
    count_nonzero_kernel<<<count_blocks(n_vox), kCountThreads, 0, s>>>(touched, n_vox, cnt);
    if ((rc = check_launch("plx_touched_count"))) return rc;
    return sync_read_u64(cnt, 1, count_out, s, "plx_touched_count");
}

}  // extern "C"

namespace plx {

int count_set_bits(const uint32_t *words, int64_t n_bits, void *ws, int64_t *count_out,
                   hipStream_t s, const char *fn) {
    if (n_bits <= 0) {
        *count_out = 0;
        return PLX_OK;
    }
    const int64_t nw = (n_bits + 31) / 32;
    auto *cnt = static_cast<unsigned long long *>(ws);
    int rc = zero_counters(ws, s, fn);
    if (rc) return rc;
    popcount_kernel<<<count_blocks(nw), kCountThreads, 0, s>>>(words, nw, n_bits, cnt);
    if ((rc = check_launch(fn))) return rc;
    return sync_read_u64(cnt, 1, count_out, s, fn);
}

}  // namespace plx
