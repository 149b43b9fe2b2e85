/*
 * plenoxel.h -- C ABI of the MI355X (gfx950) Plenoxels hot-path library.
 *
 * Plenoxels (arXiv 2112.05131) represents a radiance field as a dense index
 * grid whose cells are NULL or point into a table of occupied voxels, each
 * holding a density sigma and 27 degree-2 SH coefficients (Sec. 3.2 and
 * supplement B.1).  This library implements, in hand-written HIP kernels:
 * grid creation, density-threshold pruning with dilation and trilinear
 * resampling (Sec. 3.4), differentiable volume rendering with trilinear
 * interpolation and Max quadrature (Sec. 3.1, Eq. (1); Sec. 3.3) and its
 * exact backward pass, the TV regulariser (Sec. 3.5 and supplement B.1) and
 * RMSProp with sparse (active-voxel) updates (Sec. 3.5 and Sec. 3.8).
 *
 * General rules
 *  - Every pointer marked "device" is device memory owned by the caller.  The
 *    library never keeps a pointer after a call returns.  Pointers marked
 *    "host" are ordinary host memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All calls only
 *    enqueue work on `stream` and return, except those documented as
 *    synchronising (they return host integers and wait for `stream`).
 *  - Every call returns PLX_OK or an error code and never throws.  Arguments
 *    are validated before any launch (PLX_EINVAL); a HIP error at launch or a
 *    synchronising call is reported as PLX_EDEVICE.  plx_last_error() returns
 *    the message of the last failure on the calling thread.
 *  - The library never allocates device memory.  Calls that need scratch
 *    take a caller-owned workspace (`ws`, `ws_bytes`: device memory, 256-byte
 *    aligned, of at least the size the matching *_bytes query returns); a
 *    smaller or misaligned workspace is PLX_EINVAL before any launch.  The
 *    workspace holds nothing between calls, but two calls that share one
 *    must be ordered on a stream.
 *  - The render calls (plx_render_fwd/bwd/train/max_weight) take the ray
 *    batch's segment lists (plx_bins), made by plx_bins_count (synchronising)
 *    and plx_bins_apply (asynchronous) into caller-owned buffers; the render
 *    calls themselves neither allocate nor synchronise, so they can be
 *    captured in a graph.
 *  - Index grids are int32, z fastest: cell (i,j,k) has storage id
 *    (i*Ny + j)*Nz + k; -1 marks NULL.  Table ids of occupied voxels follow
 *    increasing storage id.
 *
 * Voxel record layout (one record per occupied voxel, table order)
 *  Logical slots 0..31: slots 0..26 are the SH coefficients, channel-major
 *  (R0..R8, G0..G8, B0..B8; basis order (l,m) = (0,0),(1,-1),(1,0),(1,1),
 *  (2,-2),(2,-1),(2,0),(2,1),(2,2)), slot 28 is the density sigma, slots 27
 *  and 29..31 are unused and kept at zero.
 *   PLX_F32  : 32 x float32 = 128 bytes (slot s at byte 4s).
 *   PLX_BF16 / PLX_F16 : 64 bytes; SH slot s (s < 27) is a 16-bit value at
 *              byte 2s, sigma is a float32 at byte 56, the rest is unused.
 *  Gradient, RMSProp state and FP32 master records always use the 128-byte
 *  PLX_F32 layout.
 */
#ifndef PLENOXEL_H
#define PLENOXEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *plx_stream; /* hipStream_t */

enum {
    PLX_OK = 0,
    PLX_EINVAL = 1,      /* bad argument; nothing was launched */
    PLX_EDEVICE = 2,     /* HIP reported an error */
    PLX_EUNSUPPORTED = 3, /* valid request this build does not implement */
    PLX_ENOMEM = 4        /* the request does not fit the fixed scratch of a
                             call that cannot allocate */
};

/* Workspace of the counting calls over a plain array (plx_mask_count,
 * plx_touched_count, plx_grid_upsample_count, plx_render_stats). */
#define PLX_COUNT_WORKSPACE_BYTES 256

enum { PLX_F32 = 0, PLX_BF16 = 1, PLX_F16 = 2 };

#define PLX_REC_SLOTS 32
#define PLX_SLOT_SIGMA 28
#define PLX_NSH 27

/* A grid as the kernels see it.  Geometry: a world point p has grid
 * coordinate g = p*scale + offset per axis (voxel centres at integers
 * 0..N-1); `step` is the sample spacing along a unit ray (world units).
 * `occ` is the occupancy structure built by plx_grid_build_occupancy
 * (plx_occ_bytes bytes; required by the render calls, ignored elsewhere). */
typedef struct plx_grid {
    int32_t reso[3];
    float scale[3];
    float offset[3];
    float step;
    int32_t sh_dtype;      /* PLX_F32 / PLX_BF16 / PLX_F16 */
    int64_t n_vox;         /* number of occupied voxels M */
    const int32_t *index;  /* device [Nx*Ny*Nz] */
    void *data;            /* device [M] records */
    const uint32_t *occ;   /* device, plx_occ_bytes(reso) bytes */
} plx_grid;

/* Options of the render calls.
 *
 * The two optional priors of Sec. 3.7 act in the gradient calls
 * (plx_render_bwd, plx_render_train, plx_render_bwd_state) on the rays of
 * the call; the other calls ignore them.  With sigma_k a sample's density
 * after the ReLU and T the ray's foreground transmittance (exp(-tau), tau its
 * optical depth):
 *   sparsity (Cauchy):  L_s = lambda_sparsity sum_{rays, samples} log(1 + 2 sigma_k^2),
 *   beta:               L_b = lambda_beta sum_rays [log(beta_eps + T) + log(beta_eps + 1 - T)].
 * Their density gradients, dL_s/dsigma_k = lambda_sparsity 4 sigma_k /
 * (1 + 2 sigma_k^2) and dL_b/dsigma_k = -delta_k T lambda_beta
 * [1/(beta_eps + T) - 1/(beta_eps + 1 - T)], pass the density ReLU and the
 * trilinear weights and are ADDED into grad with the colour gradient.  Samples
 * in cells without a non-NULL corner have density 0 and add nothing; every
 * ray adds its beta term (a miss: the constant of T = 1).  reg_loss_sum
 * (device double[2], or NULL) gets L_s and L_b ADDED.  Zero-initialise the
 * struct: zero weights turn both priors off, NULL per-ray arrays use
 * background[].  A ray's colour is C = sum_k w_k c_k + T_final bg_ray. */
typedef struct plx_render_opts {
    float background[3]; /* colour added with the transmittance left after the
                            last sample (white background of the synthetic
                            scenes, Sec. 4.1) */
    float lambda_sparsity; /* weight of the Cauchy sparsity prior (0 = off) */
    float lambda_beta;     /* weight of the beta transmittance prior (0 = off) */
    float beta_eps;        /* > 0 when lambda_beta != 0: keeps L_b finite at
                              T = 0 and T = 1 */
    double *reg_loss_sum;  /* device double[2] or NULL: (L_s, L_b) ADDED */
    const float *background_rgb; /* device [n_rays][3] or NULL: each ray's own
                                    background colour, replacing background[]
                                    (e.g. the MSI background behind it,
                                    plx_bg_render_fwd); not used by
                                    plx_render_views */
    float *grad_background;      /* device [n_rays][3] or NULL: gradient calls
                                    WRITE dL/d(background colour) = T_final
                                    dL/dC per ray (the upstream gradient of
                                    plx_bg_render_bwd) */
    void **kernel_events;        /* NULL, or 4 caller-created hipEvent_t that
                                    the binned render calls record on the
                                    stream (for timing): before the first
                                    segment kernel, after the segment
                                    forward, after the per-ray combine, and
                                    after the segment backward (the last is
                                    recorded at the end of forward-only
                                    calls too) */
} plx_render_opts;

/* ---------------------------------------------------------------- misc */

/* Message of the last failed call on this thread ("" if none). */
const char *plx_last_error(void);

/* Library version string. */
const char *plx_version(void);

/* Number of device bytes of one voxel record of dtype (128 or 64), or 0. */
int64_t plx_record_bytes(int32_t sh_dtype);

/* Number of uint32 words of the cell bitmap of a grid: 16 words (512 bits)
 * per brick of 8x8x8 cells.  Cells are indexed by their lower corner,
 * 0..N-2 per axis; there are Ba = ceil((Na-1)/8) bricks per axis, brick
 * (a,b,c) has number (a*By + b)*Bz + c, and cell (i,j,k) is bit
 * (i%8)*64 + (j%8)*8 + k%8 of the 512 bits of brick (i/8, j/8, k/8) (bit n of
 * a brick is bit n%32 of its word n/32).  Bits of cells outside the lattice
 * are 0. */
int64_t plx_occ_words(const int32_t reso[3]);

/* Bytes of the occupancy structure of a grid: the cell bitmap
 * (plx_occ_words words at offset 0) followed, at byte offset
 * plx_occ_brick_offset, by one byte per brick (brick order as above): the
 * Chebyshev distance, in bricks, to the nearest brick holding an occupied
 * cell (0 for such a brick), capped at PLX_BRICK_DIST_CAP. */
int64_t plx_occ_bytes(const int32_t reso[3]);
int64_t plx_occ_brick_offset(const int32_t reso[3]);
#define PLX_BRICK 8
#define PLX_BRICK_DIST_CAP 16

/* Grid frame of the axis-aligned box [lo, hi] (host, FP64 rounded once to
 * FP32): scale = N/(hi-lo), offset = -lo*scale - 0.5, step = step_voxels /
 * max(scale).  Voxel centres sit at grid coordinates 0..N-1. */
int plx_grid_geometry(const int32_t reso[3], const double lo[3], const double hi[3],
                      double step_voxels, float scale_out[3], float offset_out[3],
                      float *step_out);

/* Learning-rate schedule (host).  Log-linear decay from lr0 at step 0 to
 * lr1 at max_steps, times mult + (1-mult) sin(pi/2 min(1, step/delay)) when
 * delay_steps > 0: the delayed exponential of supplement B.1 (sigma) and the
 * pure exponential (SH, delay_steps = 0). */
double plx_lr_schedule(double step, double lr0, double lr1, double max_steps,
                       double delay_steps, double delay_mult);

/* ---------------------------------------------------------------- grid */

/* Bytes of workspace of the grid calls that take one (plx_grid_create,
 * plx_grid_prune_count, plx_grid_prune_weight_count, plx_grid_prune_apply,
 * plx_grid_upsample_apply) for a grid of resolution reso (for
 * plx_grid_upsample_apply: the new resolution); 0 for a bad reso.  About one
 * byte per cell. */
int64_t plx_grid_workspace_bytes(const int32_t reso[3]);

/* Number of non-zero bytes of mask[n] (device).  ws: PLX_COUNT_WORKSPACE_BYTES
 * of workspace.  Synchronising. */
int plx_mask_count(const uint8_t *mask, int64_t n, void *ws, int64_t ws_bytes, int64_t *count_out,
                   plx_stream stream);

/* Index grid from an occupancy mask (Sec. 3.2, supplement B.1): index_out[v]
 * = number of set mask bytes before v, or -1 where mask[v] == 0.  mask and
 * index_out are device arrays of Nx*Ny*Nz entries; ws: workspace of
 * plx_grid_workspace_bytes(reso). */
int plx_grid_create(const uint8_t *mask, const int32_t reso[3], int32_t *index_out, void *ws,
                    int64_t ws_bytes, plx_stream stream);

/* Writes n records of sh_dtype into out (device): density[n] and sh[n][27]
 * (device float32) when given, else the constant sigma0 and DC coefficient
 * dc (all three channels; higher orders 0).  Unused slots are zeroed and 16-bit
 * SH are rounded to nearest even. */
int plx_records_pack(int32_t sh_dtype, int64_t n, const float *density, const float *sh,
                     float sigma0, float dc, void *out, plx_stream stream);

/* Reads n records of sh_dtype back to density[n] and sh[n][27] (device
 * float32; either may be NULL). */
int plx_records_unpack(int32_t sh_dtype, int64_t n, const void *records, float *density,
                       float *sh, plx_stream stream);

/* Converts n records from src_dtype to dst_dtype (device to device; 16-bit
 * results rounded to nearest even).  src and dst must not overlap. */
int plx_records_convert(int32_t src_dtype, const void *src, int32_t dst_dtype, void *dst,
                        int64_t n, plx_stream stream);

/* Occupancy structure (layout at plx_occ_words / plx_occ_bytes): the bit of
 * cell (i,j,k) (lower corner, i < Nx-1, j < Ny-1, k < Nz-1) is set when the
 * cell has at least one non-NULL corner voxel, and each brick gets its
 * distance to the nearest brick with a set bit.  The bitmap is brick-major so
 * that the cells a ray crosses inside one brick share one 64-byte line.  A
 * sample in a cell without that bit reads only zeros and adds nothing to
 * colour, transmittance or gradient, so the render kernels skip such
 * samples, and whole boxes of empty bricks, exactly.
 * occ_out: device, plx_occ_bytes(reso) bytes.  Temporary device memory is not
 * used. */
int plx_grid_build_occupancy(const plx_grid *grid, uint32_t *occ_out, plx_stream stream);

/* Density-threshold pruning with dilation (Sec. 3.4; supplement B.1): a
 * voxel is occupied when non-NULL with stored density >= sigma_thresh; a
 * non-NULL voxel is kept when it or one of its 26 neighbours is occupied.
 * keep_out (device u8 [Nx*Ny*Nz]) gets 1 for kept voxels.  Returns the
 * numbers kept and removed (exact integers).  ws: workspace of
 * plx_grid_workspace_bytes(grid->reso).  Synchronising. */
int plx_grid_prune_count(const plx_grid *grid, float sigma_thresh, uint8_t *keep_out, void *ws,
                         int64_t ws_bytes, int64_t *n_kept, int64_t *n_pruned, plx_stream stream);

/* Weight-threshold pruning with dilation (Sec. 3.4, pruning by weight as in
 * PlenOctrees; thresholds in supplement B.1): as plx_grid_prune_count, with a
 * voxel occupied when non-NULL with wmax[id] >= w_thresh.  wmax: device
 * float32 [n_vox], the per-voxel maximum sample weight of
 * plx_render_max_weight over the training rays.  keep_out, the counts and the
 * errors are those of plx_grid_prune_count; compact with
 * plx_grid_prune_apply.  ws as plx_grid_prune_count.  Synchronising. */
int plx_grid_prune_weight_count(const plx_grid *grid, const float *wmax, float w_thresh,
                                uint8_t *keep_out, void *ws, int64_t ws_bytes, int64_t *n_kept,
                                int64_t *n_pruned, plx_stream stream);

/* Compacts a pruned grid: out->index and out->data (sized n_kept from
 * plx_grid_prune_count, same reso and dtype as grid) get the kept voxels in
 * the original order.  ws: workspace of plx_grid_workspace_bytes(grid->reso). */
int plx_grid_prune_apply(const plx_grid *grid, const uint8_t *keep, plx_grid *out, void *ws,
                         int64_t ws_bytes, plx_stream stream);

/* Number of voxels of the grid resampled to new_reso: new voxel j (per
 * axis) is occupied when its parent cell floor((2j+1) N_old / (2 N_new)) is
 * occupied.  ws: PLX_COUNT_WORKSPACE_BYTES of workspace.  Synchronising. */
int plx_grid_upsample_count(const plx_grid *grid, const int32_t new_reso[3], void *ws,
                            int64_t ws_bytes, int64_t *n_out, plx_stream stream);

/* Resamples to out->reso (Sec. 3.4: trilinear initialisation after
 * subdivision; any ratio): occupancy as in plx_grid_upsample_count, values
 * by trilinear interpolation of the old field (NULL = 0) at old grid
 * coordinate ((j + 0.5) N_old / N_new) - 0.5 clamped to [0, N_old - 1]
 * (computed in FP64).  out->data has out->sh_dtype records.  ws: workspace
 * of plx_grid_workspace_bytes(out->reso). */
int plx_grid_upsample_apply(const plx_grid *grid, plx_grid *out, void *ws, int64_t ws_bytes,
                            plx_stream stream);

/* ---------------------------------------------------------------- rays */

/* NDC warp of forward-facing rays (Sec. 3.6: forward-facing scenes use the
 * normalized device coordinates derived in the NeRF paper).  Rays are given
 * in the frame of a reference pinhole camera looking along -z (width x
 * height pixels, focal length in pixels, near plane at z = -near).  A world
 * point (x, y, z), z < 0, maps to (-(2f/W) x/z, -(2f/H) y/z, 1 + 2 near/z):
 * the near plane goes to NDC z = -1, infinity to z = +1.  Each ray is moved
 * to its point o on the near plane and becomes
 *   o' = (-(2f/W) o_x/o_z, -(2f/H) o_y/o_z, 1 + 2 near/o_z),
 *   d' = (-(2f/W)(d_x/d_z - o_x/o_z), -(2f/H)(d_y/d_z - o_y/o_z), -2 near/o_z),
 * normalised, so the render calls march it in NDC space (sample intervals
 * are NDC distances).  FP64 in that operation order without contraction,
 * rounded to FP32 once.  A ray with d_z = 0 gets origin and direction 0 (no
 * samples).  rays_o/rays_d/o_out/d_out: device float32 [n_rays][3]; the
 * outputs may alias the inputs.  Render the warped rays with a grid whose
 * box is the NDC cube [-1, 1]^3 (any per-axis resolution). */
int plx_rays_to_ndc(const float *rays_o, const float *rays_d, int64_t n_rays, int32_t width,
                    int32_t height, double focal, double near, float *o_out, float *d_out,
                    plx_stream stream);

/* ---------------------------------------------------------------- background */

/* MSI background of 360-degree scenes (Sec. 3.6, background model;
 * supplement B.1).  bg_grid is a grid of reso (L, H, W), L, H, W >= 2, with
 * FP32 records (sh_dtype PLX_F32; its geometry fields must be valid but are
 * not used): L spheres around the origin spaced linearly in inverse radius
 * (radial grid coordinate u = (1 - 1/r) L - 1/2, sphere l at u = l, so
 * 1/r = 1 - (l + 1/2)/L), each an equirectangular image of H rows (polar
 * angle theta from +z: y = theta/pi H - 1/2, clamped to [0, H-1]) and W
 * columns (azimuth phi in [0, 2 pi) from +x towards +y: x = phi/(2 pi) W - 1/2,
 * periodic).  A voxel holds an opacity density (slot 28) and one colour
 * coefficient per channel, the degree-0 SH term (slots 24, 25, 26: with the
 * density one 64-byte line of the record; other slots are not read); NULL
 * reads as zero.
 *
 * Ray samples: u_k = k/2, k = 0 .. 2(L-1)-1, at the point where the ray
 * (unit direction, origin normally inside the unit sphere) leaves the sphere
 * of that inverse radius (a sphere that does not contain the origin gives no
 * sample); trilinear interpolation of density and coefficients; opacity per
 * unit of u: alpha_k = 1 - exp(-max(0, sigma_k)/2); colour max(0, Y00 k)
 * per channel (Y00 = 1/(2 sqrt(pi))); composited as in Eq. (1) and closed
 * with the remaining transmittance times background[3] (host).  Sample
 * geometry in FP64 (no contraction), values in FP32, optical depth in FP64.
 *
 * plx_bg_render_fwd: rgb_out (device [n_rays][3]) = the background colour of
 * each ray, t_out (device [n_rays] or NULL) = its remaining transmittance.
 * Pass rgb_out as plx_render_opts.background_rgb of the foreground calls.
 * plx_bg_render_bwd: for dL/d(background colour) = grad_rgb (device
 * [n_rays][3], e.g. plx_render_opts.grad_background of the foreground
 * gradient call), ADDS the gradients of the densities and the three
 * coefficients into grad (device [M] FP32 records, slots 24-26 and 28, FP32
 * atomics) and sets
 * touched (device uint8 [M]) to 1 for every non-NULL corner of every sample
 * (both may be NULL for a background with no stored voxel). */
/* TV of the MSI background (supplement B.1: the same TV as plx_tv_grad,
 * wrapping around the edges of the equirectangular image): plx_tv_grad's
 * terms, normalisation, segment and errors, with the colour terms taken over
 * the three colour coefficients (slots 24-26, weight lambda_color) and the
 * last (azimuth) axis periodic: column W-1's neighbour is column 0.  FP32
 * records only. */
int plx_bg_tv_grad(const plx_grid *bg_grid, int64_t cell_start, int64_t cell_count,
                   float lambda_sigma, float lambda_color, float eps, float *grad, uint8_t *touched,
                   double *loss_sum, plx_stream stream);

int plx_bg_render_fwd(const plx_grid *bg_grid, const float *rays_o, const float *rays_d,
                      int64_t n_rays, const float background[3], float *rgb_out, float *t_out,
                      plx_stream stream);
int plx_bg_render_bwd(const plx_grid *bg_grid, const float *rays_o, const float *rays_d,
                      int64_t n_rays, const float background[3], const float *grad_rgb, float *grad,
                      uint8_t *touched, plx_stream stream);

/* ---------------------------------------------------------------- render */

/* Segment lists of a ray batch (the work lists of the render calls).
 *
 * The render calls process a batch in brick order: each ray is cut into
 * segments, one per 8x8x8-cell brick with an occupied cell that its samples
 * enter (Sec. 3.1-3.3 fix the samples; the cut changes only the order of
 * the work, not what is computed), and the segments are sorted by brick so
 * that rays crossing the same voxels run together.  The lists depend only on
 * the rays, the grid's geometry and its occupancy structure (not on the
 * voxel values), so one set serves every render call on those rays until the
 * occupancy is rebuilt.
 *
 * Two phases, on caller-owned device buffers (each 256-byte aligned):
 *  1. plx_bins_count fills the ray buffer (plx_bins_ray_bytes(reso, n_rays)
 *     bytes: per-ray and per-bin counts and offsets, per-bin sample counts,
 *     the list of bricks with segments, scan temporaries, a status word) and
 *     the descriptor's counts: n_seg segments, n_samp sample slots (the
 *     samples of all segments, occupied or not) and n_brick bricks with
 *     segments.  Synchronising.
 *  2. The caller attaches a segment buffer of plx_bins_seg_bytes(n_seg)
 *     bytes and, optionally, a sample buffer of
 *     plx_bins_samp_bytes(n_seg, n_samp) bytes; plx_bins_apply writes the
 *     bin-major segment records (and the segments' sample slots).
 *     Asynchronous.
 * With a sample buffer the backward pass of plx_render_bwd/plx_render_train
 * is the recorded one: the forward stores each occupied sample's position
 * and interpolated values (32 B) in the sample buffer (where the bricks
 * hold at least 40 segments on average, one workgroup per brick with the
 * samples interpolated by all its lanes from the brick's corner records in
 * LDS), and the backward runs the reverse recurrence over them
 * and sums the gradients per voxel, one brick per workgroup, so each voxel
 * receives one line of FP32 atomics per brick instead of one per segment
 * (same terms, other order of the additions).  Without one (samp_buf
 * NULL) a replay of each segment scatters its gradients itself.
 * The render calls use the buffers as their scratch (per-ray and
 * per-segment values passed between their kernels), so render calls that
 * share one plx_bins must be ordered on a stream; counting the next batch
 * into other buffers may overlap them.  plx_bins_verify (synchronising)
 * reports whether the emitting walk of plx_bins_apply met a segment the
 * count did not reserve (never expected: both walks run the same FP32
 * recipe; such a segment is dropped rather than written out of range).
 * Limits: n_rays and n_seg below 2^31 - 256, n_samp at most 2^40. */
typedef struct plx_bins {
    int64_t n_rays;        /* rays the lists were made for */
    int64_t n_seg;         /* segments */
    int64_t n_samp;        /* sample slots of the segments */
    int64_t n_brick;       /* bricks with segments */
    void *ray_buf;         /* device, ray_buf_bytes */
    int64_t ray_buf_bytes;
    void *seg_buf;         /* device, seg_buf_bytes (may be NULL when n_seg == 0) */
    int64_t seg_buf_bytes;
    void *samp_buf;        /* device, samp_buf_bytes, or NULL (optional) */
    int64_t samp_buf_bytes;
} plx_bins;

/* Bytes of the ray buffer for n_rays rays on a grid of resolution reso, of
 * the segment buffer for n_seg segments, and of the sample buffer for n_seg
 * segments with n_samp sample slots (0 for bad arguments). */
int64_t plx_bins_ray_bytes(const int32_t reso[3], int64_t n_rays);
int64_t plx_bins_seg_bytes(int64_t n_seg);
int64_t plx_bins_samp_bytes(int64_t n_seg, int64_t n_samp);

/* Phase 1: counts the segments of the rays (rays_o/rays_d: device float32
 * [n_rays][3]) into ray_buf and sets *bins to the rays, the ray buffer and
 * the three counts (segment and sample buffers NULL).  Synchronising (waits
 * for `stream`). */
int plx_bins_count(const plx_grid *grid, const float *rays_o, const float *rays_d, int64_t n_rays,
                   void *ray_buf, int64_t ray_buf_bytes, plx_bins *bins, plx_stream stream);

/* Phase 2: writes the segment records of bins->n_rays rays (the same rays and
 * grid as phase 1; bins as filled by it, with seg_buf and optionally
 * samp_buf attached) into bins->seg_buf, and their sample slots into
 * bins->samp_buf.  Asynchronous. */
int plx_bins_apply(const plx_grid *grid, const float *rays_o, const float *rays_d,
                   const plx_bins *bins, plx_stream stream);

/* PLX_OK when every segment of plx_bins_apply went where plx_bins_count
 * reserved it, PLX_EDEVICE otherwise.  Synchronising.  After a PLX_EDEVICE
 * the render calls' results on those bins are not defined (a segment
 * without sample slots contributes nothing to a training call). */
int plx_bins_verify(const plx_grid *grid, const plx_bins *bins, plx_stream stream);

/* Forward rendering (Sec. 3.1-3.3).  Each ray (unit direction) is marched
 * through the lattice hull [0,N-1]^3 at t_k = t_near + k*step while
 * t_k < t_far; sample k stands for the interval min(step, t_far - t_k).
 * sigma and the 27 SH coefficients are trilinear in the 8 surrounding
 * voxels (NULL = 0); sigma and each colour channel are clipped at 0; colour
 * is composited with Eq. (1) and the background is added with the remaining
 * transmittance.  Outputs (device float32): rgb_out[n_rays][3] and tau_out[n_rays]
 * = sum sigma_k delta_k (the optical depth, so T_final = exp(-tau)).  tau_out
 * may be NULL.  bins: the segment lists of these rays (plx_bins). */
int plx_render_fwd(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                   const float *rays_d, int64_t n_rays, const plx_bins *bins, float *rgb_out,
                   float *tau_out, plx_stream stream);

/* Backward pass of plx_render_fwd for a given dL/dC (grad_rgb[n_rays][3]).
 * Each ray is replayed from its last sample to its first with the
 * transmittance recomputed from optical depths (no per-sample state is kept
 * between the calls; tau_fwd[n_rays], the forward's optical depth, is part of
 * the forward/backward contract but this call recomputes it).  Gradients of
 * sigma and the SH coefficients are ADDED (FP32 atomics) into grad (device
 * [M] FP32 records); touched (device uint8[M], one byte per voxel) is set to 1
 * for every non-NULL corner voxel of every sample in an occupied cell (plain
 * byte stores: set bytes are never cleared here).  grad and touched may be
 * NULL when the grid has no occupied voxel (nothing is written then).
 * bins: the segment lists of these rays (plx_bins). */
int plx_render_bwd(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                   const float *rays_d, int64_t n_rays, const plx_bins *bins, const float *grad_rgb,
                   const float *tau_fwd, float *grad, uint8_t *touched, plx_stream stream);

/* One fused training pass over a ray batch: forward, the MSE reconstruction
 * loss of Sec. 3.5 with its gradient dL/dC = 2 loss_scale (C - target), and
 * the backward pass into grad/touched as in plx_render_bwd.  loss_scale is
 * 1/(number of rays of the batch) for the paper's mean; loss_sum (device
 * double, ADDED) accumulates loss_scale * sum ||C - target||^2.  rgb_out may
 * be NULL.  bins: the segment lists of these rays (plx_bins). */
int plx_render_train(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                     const float *rays_d, const float *target, int64_t n_rays,
                     const plx_bins *bins, float loss_scale, float *rgb_out, float *grad,
                     uint8_t *touched, double *loss_sum, plx_stream stream);

/* plx_render_train for callers that cannot allocate device memory or
 * synchronise (code under graph capture, tight serving or training loops):
 * the same fused forward, MSE and backward, with the same arguments and
 * results, but no plx_bins: the segment lists are built inside the call in a
 * fixed scratch array of the library's own (64 MiB per device, kept until
 * the process ends), sized for the worst case of n_rays * (Bx + By + Bz)
 * segments (Ba = bricks per axis, plx_occ_words), and the segment kernels
 * read the true count on the device.  A batch whose ray buffer
 * (plx_bins_ray_bytes) plus segment buffer for that worst case
 * (plx_bins_seg_bytes) exceeds 64 MiB is refused with PLX_ENOMEM before any
 * launch: up to 12,532 rays on a 256^3 grid, 3,350 on 512^3.
 * Never allocates or synchronises.  Every call on a device uses that
 * device's one array, and the next call overwrites it: calls that overlap
 * on one device (other streams, other threads) race; order them. */
int plx_render_train_static(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                            const float *rays_d, const float *target, int64_t n_rays,
                            float loss_scale, float *rgb_out, float *grad, uint8_t *touched,
                            double *loss_sum, plx_stream stream);

/* Per-voxel maximum sample weight, the statistic of pruning by weight
 * (Sec. 3.4, the method of PlenOctrees).  Sample k of a ray has the weight
 * w_k = T_k (1 - exp(-sigma_k delta_k)) that Eq. (1) gives its colour, with
 * the samples, densities and transmittance of plx_render_fwd (FP32 weights,
 * FP64 optical depth).  Each non-NULL corner voxel of the sample's cell (the
 * 8 voxels its interpolation reads) is raised to at least w_k:
 * wmax[id] = max(wmax[id], w_k).  wmax: device float32 [n_vox], caller-owned
 * and caller-initialised (zeros before the first batch); calls over batches
 * of rays accumulate the maximum over all of them, in any order.  Samples in
 * cells without a non-NULL corner have no voxel to raise and are skipped.
 * bins: the segment lists of these rays (plx_bins). */
int plx_render_max_weight(const plx_grid *grid, const float *rays_o, const float *rays_d,
                          int64_t n_rays, const plx_bins *bins, float *wmax, plx_stream stream);

/* Backward without recomputing the samples (the stored-state variant of the
 * backward pass of Sec. 3.1-3.3).  plx_render_fwd_state is plx_render_fwd
 * that also records, for each ray, its occupied samples in order: the sample
 * index and the pre-activation density and SH-projected colour (the colour
 * coefficients dotted with the ray's SH basis, per channel), at most `cap`
 * per ray, plus the ray's total count.  plx_render_bwd_state is
 * plx_render_bwd that replays those samples (it still reads the corner index
 * entries for the scatter, but no voxel records); a ray with more than `cap`
 * occupied samples is replayed by recomputation.  Results equal
 * plx_render_bwd's up to FP32 rounding order.
 *
 * `state` is caller-owned device memory of plx_render_state_bytes(n_rays,
 * cap) bytes, 256-byte aligned, written by the forward call and read by the
 * backward call with the same rays, grid and cap.  Layout: int32
 * count[n_rays]; int32 index[n_rays][cap]; float4 values[n_rays][cap] (each
 * part starts on a 256-byte boundary).  0 <= cap <= 2^20. */
int64_t plx_render_state_bytes(int64_t n_rays, int32_t cap);
int plx_render_fwd_state(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                         const float *rays_d, int64_t n_rays, float *rgb_out, float *tau_out,
                         void *state, int64_t state_bytes, int32_t cap, plx_stream stream);
int plx_render_bwd_state(const plx_grid *grid, const plx_render_opts *opts, const float *rays_o,
                         const float *rays_d, int64_t n_rays, const float *grad_rgb,
                         const float *tau_fwd, const void *state, int64_t state_bytes, int32_t cap,
                         float *grad, uint8_t *touched, plx_stream stream);

/* One novel-view request (serving).  Rays are pixel-centred pinhole rays:
 * pixel (px, py) of a width x height image gets, in FP64 with sums left to
 * right and then rounded to FP32, d_cam = ((px + 0.5 - width/2)/focal,
 * -((py + 0.5 - height/2)/focal), -1), d = R d_cam / |R d_cam| and o = the
 * camera centre, where c2w = [R | centre] is row-major 3x4 (columns: the
 * camera x, y, z axes and its centre; the camera looks along -z, image y
 * points up). */
typedef struct plx_view {
    double c2w[12];
    double focal;       /* pixels; principal point at the image centre */
    int32_t width;
    int32_t height;
    int32_t scene;      /* index into the scene table */
    int32_t reserved;   /* set to 0 */
    int64_t out_offset; /* index (in pixels) of this view's first pixel in rgb_out */
} plx_view;

/* Scene table: the device copy of the descriptors of n_scenes resident scenes
 * (one sh_dtype, occupancy built) that plx_render_views renders from.  Its
 * size; and the call that writes it into `table` (device, 256-byte aligned,
 * plx_scene_table_bytes bytes), asynchronously on `stream` (the descriptors
 * travel as kernel arguments: no copy engine, and the host array may be
 * released on return).  Write it again after a scene's grid changes. */
int64_t plx_scene_table_bytes(int32_t n_scenes);
int plx_scene_table_set(const plx_grid *scenes, int32_t n_scenes, void *table, int64_t table_bytes,
                        plx_stream stream);

/* Bytes of the tile queue of plx_render_views: device memory, 256-byte
 * aligned, zero-filled once before its first use (every launch leaves it at
 * zero again, apart from the sticky status word). */
#define PLX_VIEWS_QUEUE_BYTES 256

/* Renders a batch of novel views of resident scenes (the forward model of
 * plx_render_fwd, Sec. 3.1-3.3, with rays generated on the device;
 * interactive rendering is claimed in Sec. 1).  The views may mix scenes and
 * resolutions.  All pixels of all views form one queue of 16x16-pixel tiles
 * drained by a persistent grid, so the colour of a pixel depends only on its
 * ray and scene, never on the rest of the batch.  scene_table: written by
 * plx_scene_table_set for n_scenes scenes of storage type sh_dtype.  views:
 * host array, validated here (scene index, size, focal, offset) and passed
 * to the device as kernel arguments, 24 views per launch: the call
 * allocates nothing, copies nothing through a copy engine, never
 * synchronises, and the array may be released on return.  queue: the tile
 * queue (PLX_VIEWS_QUEUE_BYTES); launches that share one must be ordered on
 * a stream, launches on separate queues may overlap.  A table that is not of
 * sh_dtype (or holds fewer scenes than a view names) renders nothing for
 * those views and sets the queue's status word, which
 * plx_render_views_status reads.  rgb_out: device float32, 3 floats per
 * pixel at 3*(out_offset + py*width + px). */
int plx_render_views(const void *scene_table, int32_t n_scenes, int32_t sh_dtype, const plx_view *views,
                     int32_t n_views, const plx_render_opts *opts, float *rgb_out, void *queue,
                     plx_stream stream);

/* PLX_OK unless a launch on `queue` met a mismatched table or scene (then
 * PLX_EINVAL; the status stays set).  Synchronising. */
int plx_render_views_status(const void *queue, plx_stream stream);

/* Work counters of a ray batch, for bandwidth accounting (not timed work):
 * counts[0] = samples (all), counts[1] = samples in occupied cells,
 * counts[2] = distinct index entries read (corners of occupied cells),
 * counts[3] = distinct non-NULL voxels read.  cell_mark is device scratch of
 * ceil(Nx*Ny*Nz/32) words and vox_mark of ceil(M/32) words; both are cleared
 * by the call; ws: PLX_COUNT_WORKSPACE_BYTES of workspace.  Synchronising. */
int plx_render_stats(const plx_grid *grid, const float *rays_o, const float *rays_d,
                     int64_t n_rays, uint32_t *cell_mark, uint32_t *vox_mark, void *ws,
                     int64_t ws_bytes, int64_t counts[4], plx_stream stream);

/* ---------------------------------------------------------------- TV */

/* Total variation over cell_count cells starting at storage id cell_start
 * (wrapping modulo the number of cells; contiguous segments in storage
 * order, supplement B.1).  For cell v and channel d, Delta_a = (D_a/256)
 * (V_d(v+e_a) - V_d(v)) and term = sqrt(sum_a Delta_a^2 + eps); for sigma a
 * NULL or out-of-range neighbour reads 0, for SH a NULL current cell has no
 * terms and a NULL or out-of-range neighbour counts as equal to the current
 * cell.  Adds lambda_sigma/count * d(sum term_sigma) + lambda_sh/count *
 * d(sum term_sh) into grad (device [M] FP32 records), sets the touched byte
 * of every non-NULL voxel among v and its three forward neighbours, and ADDS the
 * loss to loss_sum (device double; may be NULL).  eps must be positive and
 * finite (PLX_EINVAL otherwise): with eps = 0 a cell whose differences all
 * vanish would have an infinite derivative. */
int plx_tv_grad(const plx_grid *grid, int64_t cell_start, int64_t cell_count,
                float lambda_sigma, float lambda_sh, float eps, float *grad,
                uint8_t *touched, double *loss_sum, plx_stream stream);

/* ---------------------------------------------------------------- optimiser */

/* Number of nonzero bytes among touched[0..n_vox) (the active set of a
 * step).  ws: PLX_COUNT_WORKSPACE_BYTES of workspace.  Synchronising. */
int plx_touched_count(const uint8_t *touched, int64_t n_vox, void *ws, int64_t ws_bytes,
                      int64_t *count_out, plx_stream stream);

/* RMSProp (Sec. 3.5) on the active voxels (nonzero touched bytes): for each
 * of the 28 values, v <- beta v + (1-beta) g^2 and p <- p - lr g / (sqrt(v) +
 * eps), lr = lr_sigma for sigma and lr_sh for SH; then g <- 0 and the touched
 * bytes are cleared.  Inactive voxels are not read or written.  vstate and
 * grad are FP32 records.  For 16-bit grids `master` holds the FP32 records
 * that are updated and grid->data receives their rounding; for PLX_F32 grids
 * master must be NULL and grid->data is updated in place. */
int plx_rmsprop_step(const plx_grid *grid, float *master, float *vstate, float *grad,
                     uint8_t *touched, float lr_sigma, float lr_sh, float beta, float eps,
                     plx_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* PLENOXEL_H */
