/*
 * plenoxel_oracle.c -- plain FP64 CPU oracle for the Plenoxels hot path
 * (Fridovich-Keil, Yu et al., "Plenoxels: Radiance Fields without Neural
 * Networks", arXiv 2112.05131).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the HIP library,
 * and it includes nothing from it.
 *
 * Precision contract.  Every *discrete* decision (ray hit/miss, number of
 * samples, the lower-corner cell of each sample, the touched set, prune and
 * upsample occupancy) follows one fixed IEEE-FP32 recipe so that an FP32 GPU
 * path can reproduce it bit for bit.  Everything continuous (interpolation,
 * SH colour, compositing, gradients, TV, RMSProp) is FP64.  The file must be
 * compiled with -ffp-contract=off so that the FP32 recipe is not fused.
 *
 * What is computed, with the passage of the paper each part follows:
 *   - data structure: dense index grid of int32, -1 = NULL, pointing into a
 *     table of (sigma, 27 SH coefficients); NULL reads as all-zero
 *     (Sec. 3.2; supplement B.1 "Implementation Details");
 *   - trilinear interpolation of sigma and SH at each sample (Sec. 3.3);
 *   - degree-2 real SH colour per channel, clipped with a ReLU (Sec. 3.2;
 *     supplement B.1, ReLU instead of a sigmoid);
 *   - Max quadrature, Eq. (1), composited over a background colour
 *     (Sec. 3.1; white background of the synthetic scenes, Sec. 4.1);
 *   - the exact gradient of Eq. (1) for a given dL/dC (chain rule written
 *     out; the paper's "gradient kernels", supplement B.1);
 *   - TV regulariser with the 256/D normalisation and the SH edge rule
 *     (Sec. 3.5, loss below Eq. (2); supplement B.1);
 *   - the Cauchy sparsity and beta transmittance priors (Sec. 3.7);
 *   - the NDC warp of rays for forward-facing scenes (Sec. 3.6);
 *   - the MSI background model of 360-degree scenes (Sec. 3.6);
 *   - RMSProp (Sec. 3.5);
 *   - density-threshold pruning with dilation, the per-voxel maximum sample
 *     weight that pruning by weight thresholds, and trilinear resampling to
 *     a new resolution (Sec. 3.4).
 * Readings where the paper is silent (sample placement, SH constants and
 * signs, sigma ReLU, TV epsilon, RMSProp beta/eps, background rule) are the
 * ones listed in the design notes; each is restated where it is used.
 *
 * Parity pins live in tests/test_oracle_*.py; every function below is pinned
 * by at least one closed form, invariant, library routine or brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* record slots of the MSI background's three colour coefficients */
#define ORC_BG_SLOT 24

#define ORC_NSH 27 /* 3 colour channels x 9 degree-2 SH coefficients */

/* Number of host threads the oracle's parallel loops use (timing runs set
 * it; results do not depend on it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Grid coordinate frame.  Voxel values live at voxel centres: voxel i of an
 * axis of N voxels spanning [lo, hi] sits at world lo + (i + 0.5) (hi-lo)/N,
 * i.e. at grid coordinate i, where g = p * scale + offset with
 * scale = N/(hi-lo) and offset = -lo*scale - 0.5.  The step along a unit ray
 * is step_voxels voxel lengths of the finest axis.  FP64 maths, rounded to
 * FP32 once. */
void orc_grid_geometry(const int32_t reso[3], const double lo[3],
                       const double hi[3], double step_voxels,
                       float scale_out[3], float offset_out[3],
                       float *step_out)
{
    double max_scale = 0.0;
    for (int a = 0; a < 3; ++a) {
        double s = (double)reso[a] / (hi[a] - lo[a]);
        scale_out[a] = (float)s;
        offset_out[a] = (float)(-lo[a] * s - 0.5);
        if (s > max_scale) max_scale = s;
    }
    *step_out = (float)(step_voxels / max_scale);
}

/* ------------------------------------------------------------------------ */
/* FP32 ray/sample recipe (discrete decisions). */

typedef struct {
    float og[3], dg[3];
    float t_near, t_far;
} ray_geom;

/* Slab test of the ray against the lattice hull [0, N-1]^3 in grid
 * coordinates.  Returns 1 on a hit (t_near < t_far), 0 on a miss. */
static int ray_setup(const int32_t reso[3], const float scale[3],
                     const float offset[3], const float o[3], const float d[3],
                     ray_geom *r)
{
    float t_near = 0.0f;
    float t_far = INFINITY;
    for (int a = 0; a < 3; ++a) {
        float og = o[a] * scale[a];
        og = og + offset[a];
        float dg = d[a] * scale[a];
        float top = (float)(reso[a] - 1);
        r->og[a] = og;
        r->dg[a] = dg;
        if (dg == 0.0f) {
            if (og < 0.0f || og > top) return 0;
            continue;
        }
        float t0 = (-og) / dg;
        float t1 = (top - og) / dg;
        float tlo = t0 < t1 ? t0 : t1;
        float thi = t0 < t1 ? t1 : t0;
        if (tlo > t_near) t_near = tlo;
        if (thi < t_far) t_far = thi;
    }
    r->t_near = t_near;
    r->t_far = t_far;
    /* a zero direction has no exit point: no samples */
    if (!(t_far < INFINITY)) return 0;
    return t_near < t_far;
}

/* Parameter of sample k: computed directly from k, never by accumulation. */
static float sample_t(const ray_geom *r, float step, int k)
{
    float kk = (float)k * step;
    return r->t_near + kk;
}

/* Lower-corner cell and in-cell fraction of the sample at parameter t. */
static void sample_cell(const int32_t reso[3], const ray_geom *r, float t,
                        int cell[3], double frac[3])
{
    for (int a = 0; a < 3; ++a) {
        float p = t * r->dg[a];
        float g = r->og[a] + p;
        int i0 = (int)floorf(g);
        if (i0 < 0) i0 = 0;
        if (i0 > reso[a] - 2) i0 = reso[a] - 2;
        float f = g - (float)i0;
        if (f < 0.0f) f = 0.0f;
        if (f > 1.0f) f = 1.0f;
        cell[a] = i0;
        frac[a] = (double)f;
    }
}

/* Length of the interval that sample k stands for: the step, except the last
 * interval, which stops at the exit point t_far (left-endpoint samples,
 * "constant values between samples", Sec. 3.1). */
static float sample_delta(const ray_geom *r, float step, float t)
{
    float rest = r->t_far - t;
    return rest < step ? rest : step;
}

/* ------------------------------------------------------------------------ */
/* Degree-2 real spherical harmonics (Sec. 3.2: 9 coefficients per channel).
 * Orthonormal real basis in the order (l,m) = (0,0),(1,-1),(1,0),(1,1),
 * (2,-2),(2,-1),(2,0),(2,1),(2,2), built from the complex harmonics with the
 * Condon-Shortley phase as sqrt(2) Im Y_l^|m| (m<0), Y_l^0, sqrt(2) Re Y_l^m
 * (m>0), evaluated at the ray direction d = (x, y, z). */
void orc_sh_basis(const double d[3], double y[9])
{
    const double pi = 3.14159265358979323846;
    const double x = d[0], yy = d[1], z = d[2];
    const double c00 = 0.5 / sqrt(pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2 = sqrt(15.0 / (4.0 * pi));
    const double c20 = sqrt(5.0 / (16.0 * pi));
    const double c22 = sqrt(15.0 / (16.0 * pi));
    y[0] = c00;
    y[1] = -c1 * yy;
    y[2] = c1 * z;
    y[3] = -c1 * x;
    y[4] = c2 * x * yy;
    y[5] = -c2 * yy * z;
    y[6] = c20 * (3.0 * z * z - 1.0);
    y[7] = -c2 * x * z;
    y[8] = c22 * (x * x - yy * yy);
}

/* ------------------------------------------------------------------------ */
/* Trilinear interpolation of sigma and the 27 SH coefficients from the 8
 * voxels around a sample (Sec. 3.3).  NULL voxels read as zero (supplement
 * B.1).  Also returns the 8 corner table ids (-1 = NULL) and weights. */

static int64_t lin_id(const int32_t reso[3], int i, int j, int k)
{
    return ((int64_t)i * reso[1] + j) * (int64_t)reso[2] + k;
}

static void interpolate(const int32_t reso[3], const int32_t *index,
                        const double *density, const double *sh,
                        const int cell[3], const double f[3],
                        double *sigma, double k[ORC_NSH], int64_t ids[8],
                        double w[8])
{
    *sigma = 0.0;
    for (int q = 0; q < ORC_NSH; ++q) k[q] = 0.0;
    for (int c = 0; c < 8; ++c) {
        int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
        double wc = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                    (dz ? f[2] : 1.0 - f[2]);
        int64_t id = index[lin_id(reso, cell[0] + dx, cell[1] + dy,
                                  cell[2] + dz)];
        ids[c] = id;
        w[c] = wc;
        if (id < 0) continue;
        *sigma += wc * density[id];
        for (int q = 0; q < ORC_NSH; ++q) k[q] += wc * sh[id * ORC_NSH + q];
    }
}

/* ------------------------------------------------------------------------ */
/* Per-sample record of one ray (forward quantities the gradient needs). */
typedef struct {
    double sigma_pre;      /* interpolated sigma before the ReLU */
    double rgb_pre[3];     /* SH colour before the ReLU */
    double sigma, rgb[3];  /* after the ReLUs */
    double delta;          /* interval length */
    double T;              /* transmittance before the sample */
    double T_next;         /* transmittance after the sample */
    double weight;         /* T * (1 - exp(-sigma delta)) */
    int64_t ids[8];
    double w[8];
} sample_rec;

/* Walks one ray and fills recs (if non-NULL, capacity cap).  Returns the
 * number of samples n; *rgb and *tau get the composited colour (with the
 * background) and the optical depth sum(sigma delta). */
static int march_ray(const int32_t reso[3], const float scale[3],
                     const float offset[3], float step, const int32_t *index,
                     const double *density, const double *sh, const float o[3],
                     const float d[3], const double bg[3], sample_rec *recs,
                     int cap, double rgb[3], double *tau, double *t_final)
{
    ray_geom r;
    rgb[0] = rgb[1] = rgb[2] = 0.0;
    *tau = 0.0;
    *t_final = 1.0;
    if (!ray_setup(reso, scale, offset, o, d, &r)) {
        for (int c = 0; c < 3; ++c) rgb[c] = bg[c];
        return 0;
    }
    double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
    double ylm[9];
    orc_sh_basis(dd, ylm);

    double T = 1.0;
    int n = 0;
    for (int k = 0;; ++k) {
        float t = sample_t(&r, step, k);
        if (!(t < r.t_far)) break;
        int cell[3];
        double f[3];
        sample_cell(reso, &r, t, cell, f);
        double delta = (double)sample_delta(&r, step, t);

        double sig, kc[ORC_NSH];
        int64_t ids[8];
        double w[8];
        interpolate(reso, index, density, sh, cell, f, &sig, kc, ids, w);

        double sigma = sig > 0.0 ? sig : 0.0;
        double col_pre[3], col[3];
        for (int ch = 0; ch < 3; ++ch) {
            double s = 0.0;
            for (int l = 0; l < 9; ++l) s += kc[ch * 9 + l] * ylm[l];
            col_pre[ch] = s;
            col[ch] = s > 0.0 ? s : 0.0;
        }
        double alpha = -expm1(-sigma * delta);
        double weight = T * alpha;
        double T_next = T * exp(-sigma * delta);
        for (int ch = 0; ch < 3; ++ch) rgb[ch] += weight * col[ch];
        *tau += sigma * delta;

        if (recs && n < cap) {
            sample_rec *s = &recs[n];
            s->sigma_pre = sig;
            s->sigma = sigma;
            for (int ch = 0; ch < 3; ++ch) {
                s->rgb_pre[ch] = col_pre[ch];
                s->rgb[ch] = col[ch];
            }
            s->delta = delta;
            s->T = T;
            s->T_next = T_next;
            s->weight = weight;
            memcpy(s->ids, ids, sizeof(ids));
            memcpy(s->w, w, sizeof(w));
        }
        T = T_next;
        ++n;
    }
    for (int ch = 0; ch < 3; ++ch) rgb[ch] += T * bg[ch];
    *t_final = T;
    return n;
}

/* Number of samples of a ray (FP32 recipe only). */
static int count_samples(const int32_t reso[3], const float scale[3],
                         const float offset[3], float step, const float o[3],
                         const float d[3])
{
    ray_geom r;
    if (!ray_setup(reso, scale, offset, o, d, &r)) return 0;
    int n = 0;
    while (sample_t(&r, step, n) < r.t_far) ++n;
    return n;
}

/* ------------------------------------------------------------------------ */
/* Forward rendering of n_rays rays: rgb_out[3R], tau_out[R] (optical depth),
 * tfinal_out[R] (transmittance left after the last sample), nsamp_out[R]
 * (number of samples).  Any output may be NULL.  The background colour of
 * ray r is bg[bg_stride * r .. + 2]: bg_stride 0 gives every ray bg[0..2],
 * 3 gives each ray its own (e.g. the MSI background behind it). */
void orc_render_fwd(const int32_t reso[3], const float scale[3],
                    const float offset[3], float step, const int32_t *index,
                    const double *density, const double *sh,
                    const float *rays_o, const float *rays_d, int64_t n_rays,
                    const double *bg, int64_t bg_stride, double *rgb_out, double *tau_out,
                    double *tfinal_out, int32_t *nsamp_out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < n_rays; ++r) {
        double rgb[3], tau, tf;
        int n = march_ray(reso, scale, offset, step, index, density, sh,
                          rays_o + 3 * r, rays_d + 3 * r, bg + bg_stride * r, NULL, 0, rgb,
                          &tau, &tf);
        if (rgb_out)
            for (int c = 0; c < 3; ++c) rgb_out[3 * r + c] = rgb[c];
        if (tau_out) tau_out[r] = tau;
        if (tfinal_out) tfinal_out[r] = tf;
        if (nsamp_out) nsamp_out[r] = n;
    }
}

/* Per-sample trace of one ray, for tests: writes up to cap samples of
 * t, delta, sigma_pre, rgb_pre (3 per sample) and lower-corner cell (3 per
 * sample).  Returns the number of samples of the ray. */
int orc_trace_ray(const int32_t reso[3], const float scale[3],
                  const float offset[3], float step, const int32_t *index,
                  const double *density, const double *sh, const float o[3],
                  const float d[3], int cap, double *t_out, double *delta_out,
                  double *sigma_pre_out, double *rgb_pre_out, int32_t *cell_out)
{
    ray_geom r;
    if (!ray_setup(reso, scale, offset, o, d, &r)) return 0;
    double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
    double ylm[9];
    orc_sh_basis(dd, ylm);
    int n = 0;
    for (int k = 0;; ++k) {
        float t = sample_t(&r, step, k);
        if (!(t < r.t_far)) break;
        if (n < cap) {
            int cell[3];
            double f[3], sig, kc[ORC_NSH], w[8];
            int64_t ids[8];
            sample_cell(reso, &r, t, cell, f);
            interpolate(reso, index, density, sh, cell, f, &sig, kc, ids, w);
            t_out[n] = (double)t;
            delta_out[n] = (double)sample_delta(&r, step, t);
            sigma_pre_out[n] = sig;
            for (int ch = 0; ch < 3; ++ch) {
                double s = 0.0;
                for (int l = 0; l < 9; ++l) s += kc[ch * 9 + l] * ylm[l];
                rgb_pre_out[3 * n + ch] = s;
            }
            for (int a = 0; a < 3; ++a) cell_out[3 * n + a] = cell[a];
        }
        ++n;
    }
    return n;
}

/* Rays of a novel-view request: a pixel-centred pinhole camera of W x H
 * pixels, focal length f (pixels, principal point at the image centre) and
 * camera-to-world matrix c2w (3x4 row-major: columns are the camera x, y, z
 * axes and the centre; the camera looks along -z, image y points up).
 * Pixel (px, py), row-major, gets
 *   d_cam = ((px + 0.5 - W/2)/f, -((py + 0.5 - H/2)/f), -1),
 *   d = R d_cam / |R d_cam|  (FP64, sums left to right, rounded to FP32),
 *   o = the camera centre (rounded to FP32). */
void orc_camera_rays(const double c2w[12], double focal, int32_t width,
                     int32_t height, float *rays_o, float *rays_d)
{
    for (int32_t py = 0; py < height; ++py)
        for (int32_t px = 0; px < width; ++px) {
            double x = ((double)px + 0.5 - 0.5 * (double)width) / focal;
            double y = -(((double)py + 0.5 - 0.5 * (double)height) / focal);
            double z = -1.0;
            double dv[3];
            for (int a = 0; a < 3; ++a)
                dv[a] = c2w[4 * a + 0] * x + c2w[4 * a + 1] * y + c2w[4 * a + 2] * z;
            double nrm = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            int64_t r = (int64_t)py * width + px;
            for (int a = 0; a < 3; ++a) {
                rays_d[3 * r + a] = (float)(dv[a] / nrm);
                rays_o[3 * r + a] = (float)c2w[4 * a + 3];
            }
        }
}

/* Normalized device coordinates of forward-facing scenes (Sec. 3.6 and the
 * forward-facing experiments: the NDC space derived in the NeRF paper).
 * Rays are given in the frame of a reference pinhole camera that looks
 * along -z (width x height pixels, focal length f in pixels) with its near
 * plane at z = -near.  A world point (x, y, z), z < 0, maps to
 *   (-(2f/W) x/z, -(2f/H) y/z, 1 + 2 near/z),
 * which sends the near plane to NDC z = -1 and infinity to z = +1, and maps
 * straight lines to straight lines.  A ray is first moved to its point on
 * the near plane, o + t d with t = -(near + o_z)/d_z; with that point o:
 *   o' = (-(2f/W) o_x/o_z, -(2f/H) o_y/o_z, 1 + 2 near/o_z),
 *   d' = (-(2f/W)(d_x/d_z - o_x/o_z), -(2f/H)(d_y/d_z - o_y/o_z), -2 near/o_z),
 * and d' is normalised (the renderer marches unit directions; distances,
 * hence the sample intervals, are measured in NDC space).  FP64 with this
 * operation order, rounded to FP32 once.  A ray with d_z = 0 never reaches
 * the near plane: it gets origin and direction 0 (no samples). */
void orc_rays_to_ndc(const float *rays_o, const float *rays_d, int64_t n_rays,
                     int32_t width, int32_t height, double focal, double near,
                     float *o_out, float *d_out)
{
    const double ax = -(2.0 * focal / (double)width);
    const double ay = -(2.0 * focal / (double)height);
    for (int64_t r = 0; r < n_rays; ++r) {
        double o[3], d[3];
        for (int a = 0; a < 3; ++a) {
            o[a] = (double)rays_o[3 * r + a];
            d[a] = (double)rays_d[3 * r + a];
        }
        if (d[2] == 0.0) {
            for (int a = 0; a < 3; ++a) o_out[3 * r + a] = d_out[3 * r + a] = 0.0f;
            continue;
        }
        double t = -(near + o[2]) / d[2];
        for (int a = 0; a < 3; ++a) o[a] = o[a] + t * d[a];
        double op[3], dp[3];
        op[0] = ax * (o[0] / o[2]);
        op[1] = ay * (o[1] / o[2]);
        op[2] = 1.0 + 2.0 * near / o[2];
        dp[0] = ax * (d[0] / d[2] - o[0] / o[2]);
        dp[1] = ay * (d[1] / d[2] - o[1] / o[2]);
        dp[2] = -2.0 * near / o[2];
        double nrm = sqrt(dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2]);
        for (int a = 0; a < 3; ++a) {
            o_out[3 * r + a] = (float)op[a];
            d_out[3 * r + a] = (float)(dp[a] / nrm);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* MSI background of 360-degree scenes (Sec. 3.6, background model;
 * supplement B.1).  A grid of reso = (L, H, W): L spheres around the origin,
 * each an equirectangular image of H rows (polar angle theta from +z) and W
 * columns (azimuth phi from +x towards +y), values at cell centres as in the
 * foreground grid.  The radial grid coordinate is linear in inverse radius:
 * u = (1 - 1/r) L - 0.5, so sphere l (u = l) has 1/r = 1 - (l + 1/2)/L,
 * from just outside the unit sphere to far away (reading of the design
 * notes).  Each voxel holds an opacity density and an RGB colour (only the
 * degree-0 SH coefficient of each channel, kept in sh slots 24, 25, 26 of
 * the record, next to the density; the others are ignored); NULL reads as
 * zero.
 *
 * Samples of a ray (unit direction d, origin o inside the unit sphere): at
 * u_k = k/2 for k = 0 .. 2(L-1)-1, at the point where the ray leaves the
 * sphere of that inverse radius; a sample whose sphere does not contain o
 * has no point in front and is skipped.  At the point p: phi = atan2(p_y,
 * p_x) in [0, 2 pi), theta = acos(p_z/|p|), grid coordinates
 * gx = phi/(2 pi) W - 1/2 (periodic: column W is column 0),
 * gy = theta/pi H - 1/2 (clamped to [0, H-1] like the foreground lattice),
 * gu = u_k; trilinear interpolation over the 8 surrounding voxels.
 * Opacities are per unit of u (reading): alpha_k = 1 - exp(-sigma_k / 2),
 * sigma_k = max(0, interpolated density), colour c = max(0, Y00 k) per
 * channel (Y00 = 1/(2 sqrt(pi))), composited as in Eq. (1) and closed with
 * the remaining transmittance times bg.  FP64 throughout. */

#define ORC_Y00 0.28209479177387814
#define ORC_PI 3.14159265358979323846

typedef struct {
    int64_t ids[8];
    double w[8];
} bg_sample_t;

/* Corners and weights of background sample k; returns 0 when skipped. */
static int bg_sample(const int32_t reso[3], const int32_t *index, const double o[3],
                     const double d[3], int k, bg_sample_t *s)
{
    const int L = reso[0], H = reso[1], W = reso[2];
    double u = 0.5 * k;
    double inv_r = 1.0 - (u + 0.5) / (double)L;
    double r = 1.0 / inv_r;
    double b = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    double c = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - r * r;
    if (!(c < 0.0)) return 0;
    double t = -b + sqrt(b * b - c);
    double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    double pr = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    double cz = p[2] / pr;
    cz = cz < -1.0 ? -1.0 : (cz > 1.0 ? 1.0 : cz);
    double theta = acos(cz);
    double phi = atan2(p[1], p[0]);
    if (phi < 0.0) phi += 2.0 * ORC_PI;
    double gx = phi / (2.0 * ORC_PI) * (double)W - 0.5;
    double gy = theta / ORC_PI * (double)H - 0.5;
    double fx0 = floor(gx);
    double fx = gx - fx0;
    int x0 = (int)fx0;
    x0 = ((x0 % W) + W) % W;
    int x1 = (x0 + 1) % W;
    gy = gy < 0.0 ? 0.0 : (gy > (double)(H - 1) ? (double)(H - 1) : gy);
    int y0 = (int)floor(gy);
    if (y0 > H - 2) y0 = H - 2;
    double fy = gy - y0;
    int l0 = (int)floor(u);
    if (l0 > L - 2) l0 = L - 2;
    double fl = u - l0;
    for (int cc = 0; cc < 8; ++cc) {
        int dl = (cc >> 2) & 1, dy = (cc >> 1) & 1, dx = cc & 1;
        int64_t cell = ((int64_t)(l0 + dl) * H + (y0 + dy)) * W + (dx ? x1 : x0);
        s->ids[cc] = index[cell];
        s->w[cc] = (dl ? fl : 1.0 - fl) * (dy ? fy : 1.0 - fy) * (dx ? fx : 1.0 - fx);
    }
    return 1;
}

/* Background colour of each ray: rgb_out[3R] = sum_k w_k c_k + T bg;
 * t_out[R] (may be NULL) = the transmittance T left after the last sample. */
void orc_bg_render_fwd(const int32_t reso[3], const int32_t *index, const double *density,
                       const double *sh, const float *rays_o, const float *rays_d,
                       int64_t n_rays, const double bg[3], double *rgb_out, double *t_out)
{
    const int L = reso[0];
    for (int64_t r = 0; r < n_rays; ++r) {
        double o[3], d[3];
        for (int a = 0; a < 3; ++a) {
            o[a] = (double)rays_o[3 * r + a];
            d[a] = (double)rays_d[3 * r + a];
        }
        double T = 1.0, C[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 2 * (L - 1); ++k) {
            bg_sample_t s;
            if (!bg_sample(reso, index, o, d, k, &s)) continue;
            double sig = 0.0, kc[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 8; ++c) {
                if (s.ids[c] < 0) continue;
                sig += s.w[c] * density[s.ids[c]];
                for (int ch = 0; ch < 3; ++ch) kc[ch] += s.w[c] * sh[s.ids[c] * ORC_NSH + ORC_BG_SLOT + ch];
            }
            double sigma = sig > 0.0 ? sig : 0.0;
            double alpha = -expm1(-0.5 * sigma);
            for (int ch = 0; ch < 3; ++ch) {
                double col = ORC_Y00 * kc[ch];
                C[ch] += T * alpha * (col > 0.0 ? col : 0.0);
            }
            T *= exp(-0.5 * sigma);
        }
        for (int ch = 0; ch < 3; ++ch) rgb_out[3 * r + ch] = C[ch] + T * bg[ch];
        if (t_out) t_out[r] = T;
    }
}

/* Gradient of the background colours for a given dL/dC_bg (grad_rgb[3R]),
 * by the same chain rule as orc_render_bwd (R_k = what the ray collects
 * after sample k, T_k before it):
 *   dC/dsigma_k = (1/2)(T_{k+1} c_k - R_k),  dC/dc_k = w_k.
 * ADDED into grad_density[M] and grad_sh[M*27] (slots 24, 25, 26 only);
 * touched[M] = 1 for every non-NULL corner of every sample.
 * With gate_rel >= 0 the call instead ADDS the absolute sizes of the terms
 * (for tolerances, as orc_render_bwd_mass: grad_rgb holds |dL/dC|, the
 * density term counts as (1/2)(T_{k+1} g.c + g.R), and a term behind a
 * ReLU gate within gate_rel times its absolute sum of the kink counts as
 * open); gate_rel < 0 gives the gradient. */
void orc_bg_render_bwd(const int32_t reso[3], const int32_t *index, const double *density,
                       const double *sh, const float *rays_o, const float *rays_d,
                       int64_t n_rays, const double bg[3], const double *grad_rgb,
                       double gate_rel, double *grad_density, double *grad_sh, uint8_t *touched)
{
    const int absolute = gate_rel >= 0.0;
    const int L = reso[0];
    const int n_max = 2 * (L - 1);
    bg_sample_t *smp = (bg_sample_t *)malloc(sizeof(bg_sample_t) * (size_t)n_max);
    double *sg = (double *)malloc(sizeof(double) * (size_t)n_max * 9);
    for (int64_t r = 0; r < n_rays; ++r) {
        double o[3], d[3];
        for (int a = 0; a < 3; ++a) {
            o[a] = (double)rays_o[3 * r + a];
            d[a] = (double)rays_d[3 * r + a];
        }
        const double *g = grad_rgb + 3 * r;
        /* forward, keeping each sample's values */
        int n = 0;
        double *sig_pre = sg, *col_pre = sg + n_max, *Tk = sg + 4 * n_max;
        double *abs_sig = sg + 5 * n_max, *abs_col = sg + 6 * n_max;
        double T = 1.0;
        for (int k = 0; k < n_max; ++k) {
            if (!bg_sample(reso, index, o, d, k, &smp[n])) continue;
            double sig = 0.0, kc[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 8; ++c) {
                int64_t id = smp[n].ids[c];
                if (id < 0) continue;
                sig += smp[n].w[c] * density[id];
                for (int ch = 0; ch < 3; ++ch) kc[ch] += smp[n].w[c] * sh[id * ORC_NSH + ORC_BG_SLOT + ch];
            }
            sig_pre[n] = sig;
            for (int ch = 0; ch < 3; ++ch) col_pre[3 * n + ch] = ORC_Y00 * kc[ch];
            double as = 0.0, ac[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 8; ++c) {
                int64_t id = smp[n].ids[c];
                if (id < 0) continue;
                as += smp[n].w[c] * fabs(density[id]);
                for (int ch = 0; ch < 3; ++ch) ac[ch] += smp[n].w[c] * ORC_Y00 * fabs(sh[id * ORC_NSH + ORC_BG_SLOT + ch]);
            }
            abs_sig[n] = as;
            for (int ch = 0; ch < 3; ++ch) abs_col[3 * n + ch] = ac[ch];
            Tk[n] = T;
            T *= exp(-0.5 * (sig > 0.0 ? sig : 0.0));
            ++n;
        }
        double R[3];
        for (int ch = 0; ch < 3; ++ch) R[ch] = T * (absolute ? fabs(bg[ch]) : bg[ch]);
        for (int j = n - 1; j >= 0; --j) {
            double sigma = sig_pre[j] > 0.0 ? sig_pre[j] : 0.0;
            double T_next = Tk[j] * exp(-0.5 * sigma);
            double w = Tk[j] * -expm1(-0.5 * sigma);
            double gc = 0.0, gR = 0.0, col[3];
            int col_on[3];
            for (int ch = 0; ch < 3; ++ch) {
                double pre = col_pre[3 * j + ch];
                col[ch] = pre > 0.0 ? pre : 0.0;
                col_on[ch] = pre > 0.0 || (absolute && fabs(pre) <= gate_rel * abs_col[3 * j + ch]);
                gc += g[ch] * col[ch];
                gR += g[ch] * R[ch];
            }
            int sig_on = sig_pre[j] > 0.0 || (absolute && fabs(sig_pre[j]) <= gate_rel * abs_sig[j]);
            double dsig = sig_on ? 0.5 * (absolute ? T_next * gc + gR : T_next * gc - gR) : 0.0;
            for (int c = 0; c < 8; ++c) {
                int64_t id = smp[j].ids[c];
                if (id < 0) continue;
                touched[id] = 1;
                grad_density[id] += smp[j].w[c] * dsig;
                for (int ch = 0; ch < 3; ++ch)
                    if (col_on[ch])
                        grad_sh[id * ORC_NSH + ORC_BG_SLOT + ch] += smp[j].w[c] * w * g[ch] * ORC_Y00;
            }
            for (int ch = 0; ch < 3; ++ch) R[ch] += w * col[ch];
        }
    }
    free(sg);
    free(smp);
}

/* Ray setup only, for tests: t_near/t_far of the FP32 recipe and the sample
 * count.  Returns 1 on hit. */
int orc_ray_extent(const int32_t reso[3], const float scale[3],
                   const float offset[3], float step, const float o[3],
                   const float d[3], float *t_near, float *t_far,
                   int32_t *n_samples)
{
    ray_geom r;
    int hit = ray_setup(reso, scale, offset, o, d, &r);
    *t_near = hit ? r.t_near : 0.0f;
    *t_far = hit ? r.t_far : 0.0f;
    *n_samples = count_samples(reso, scale, offset, step, o, d);
    return hit;
}

/* ------------------------------------------------------------------------ */
/* Deterministic accumulation of per-voxel sums over rays.
 *
 * Each ray's terms are first summed per voxel, sample after sample, in a
 * private sparse accumulator (a slot per voxel the ray touches); the rays'
 * sums are then added into the output arrays in ray order.  Every voxel's
 * sum is therefore formed in one fixed order -- per ray in sample order,
 * then over the rays in batch order -- whatever the number of threads or
 * their scheduling, and the results are the same bits from run to run.
 * OpenMP runs the rays of a wave of ORC_RAY_WAVE rays in parallel (each
 * thread appends its rays' sums to its own arena), then adds the wave into
 * the outputs with the voxels split among the threads. */
#define ORC_RAY_WAVE 8192
#define ORC_ACC_W (ORC_NSH + 1) /* 27 SH values, then sigma */

typedef struct {
    int32_t *slot;   /* [M]: row of a voxel for the current ray, -1 if none */
    int64_t *ids;    /* voxels in first-touch order */
    double *val;     /* [n][ORC_ACC_W] */
    int64_t n, cap;
    /* arena of finished rays' rows for the current wave */
    int64_t *a_ids;
    double *a_val;
    int64_t a_n, a_cap;
} sparse_acc;

static void acc_init(sparse_acc *a, int64_t n_vox)
{
    a->slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_vox > 0 ? n_vox : 1));
    for (int64_t i = 0; i < n_vox; ++i) a->slot[i] = -1;
    a->cap = 1024;
    a->n = 0;
    a->ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)a->cap);
    a->val = (double *)malloc(sizeof(double) * ORC_ACC_W * (size_t)a->cap);
    a->a_cap = 4096;
    a->a_n = 0;
    a->a_ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)a->a_cap);
    a->a_val = (double *)malloc(sizeof(double) * ORC_ACC_W * (size_t)a->a_cap);
}

static void acc_free(sparse_acc *a)
{
    free(a->slot);
    free(a->ids);
    free(a->val);
    free(a->a_ids);
    free(a->a_val);
}

/* Row of voxel id for the current ray, created (zeroed) on first touch. */
static double *acc_row(sparse_acc *a, int64_t id)
{
    int32_t k = a->slot[id];
    if (k < 0) {
        if (a->n == a->cap) {
            a->cap *= 2;
            a->ids = (int64_t *)realloc(a->ids, sizeof(int64_t) * (size_t)a->cap);
            a->val = (double *)realloc(a->val, sizeof(double) * ORC_ACC_W * (size_t)a->cap);
        }
        k = (int32_t)a->n++;
        a->slot[id] = k;
        a->ids[k] = id;
        memset(a->val + (size_t)k * ORC_ACC_W, 0, sizeof(double) * ORC_ACC_W);
    }
    return a->val + (size_t)k * ORC_ACC_W;
}

/* Moves the current ray's rows to the arena; returns their first arena row. */
static int64_t acc_finish_ray(sparse_acc *a)
{
    const int64_t first = a->a_n;
    if (a->a_n + a->n > a->a_cap) {
        while (a->a_n + a->n > a->a_cap) a->a_cap *= 2;
        a->a_ids = (int64_t *)realloc(a->a_ids, sizeof(int64_t) * (size_t)a->a_cap);
        a->a_val = (double *)realloc(a->a_val, sizeof(double) * ORC_ACC_W * (size_t)a->a_cap);
    }
    memcpy(a->a_ids + a->a_n, a->ids, sizeof(int64_t) * (size_t)a->n);
    memcpy(a->a_val + (size_t)a->a_n * ORC_ACC_W, a->val, sizeof(double) * ORC_ACC_W * (size_t)a->n);
    a->a_n += a->n;
    for (int64_t k = 0; k < a->n; ++k) a->slot[a->ids[k]] = -1;
    a->n = 0;
    return first;
}

typedef void (*ray_body_fn)(const void *ctx, int64_t r, sparse_acc *acc);

/* Runs body over every ray and adds the rays' per-voxel sums into the
 * outputs in ray order (see above). */
static void accumulate_over_rays(int64_t n_rays, int64_t n_vox, ray_body_fn body, const void *ctx,
                                 double *out_density, double *out_sh, uint8_t *touched)
{
    int n_thr = 1;
#ifdef _OPENMP
    n_thr = omp_get_max_threads();
#endif
    sparse_acc *acc = (sparse_acc *)malloc(sizeof(sparse_acc) * (size_t)n_thr);
    for (int t = 0; t < n_thr; ++t) acc_init(&acc[t], n_vox);
    /* per ray of a wave: arena (thread), first row, row count */
    int32_t *r_thr = (int32_t *)malloc(sizeof(int32_t) * ORC_RAY_WAVE);
    int64_t *r_first = (int64_t *)malloc(sizeof(int64_t) * ORC_RAY_WAVE);
    int64_t *r_cnt = (int64_t *)malloc(sizeof(int64_t) * ORC_RAY_WAVE);
    for (int64_t w0 = 0; w0 < n_rays; w0 += ORC_RAY_WAVE) {
        const int64_t nw = n_rays - w0 < ORC_RAY_WAVE ? n_rays - w0 : ORC_RAY_WAVE;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < nw; ++i) {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            body(ctx, w0 + i, &acc[t]);
            r_thr[i] = t;
            const int64_t cnt = acc[t].n;
            r_first[i] = acc_finish_ray(&acc[t]);
            r_cnt[i] = cnt;
        }
        /* the wave's rays in ray order; each thread adds the rows of its
         * own share of the voxels */
#pragma omp parallel for schedule(static, 1)
        for (int part = 0; part < n_thr; ++part) {
            for (int64_t i = 0; i < nw; ++i) {
                const sparse_acc *a = &acc[r_thr[i]];
                for (int64_t k = r_first[i]; k < r_first[i] + r_cnt[i]; ++k) {
                    const int64_t id = a->a_ids[k];
                    if (id % n_thr != part) continue;
                    const double *v = a->a_val + (size_t)k * ORC_ACC_W;
                    for (int q = 0; q < ORC_NSH; ++q) out_sh[id * ORC_NSH + q] += v[q];
                    out_density[id] += v[ORC_NSH];
                    if (touched) touched[id] = 1;
                }
            }
        }
        for (int t = 0; t < n_thr; ++t) acc[t].a_n = 0;
    }
    free(r_thr);
    free(r_first);
    free(r_cnt);
    for (int t = 0; t < n_thr; ++t) acc_free(&acc[t]);
    free(acc);
}

typedef struct {
    const int32_t *reso;
    const float *scale, *offset;
    float step;
    const int32_t *index;
    const double *density, *sh;
    const float *rays_o, *rays_d;
    const double *bg;
    int64_t bg_stride;
    const double *g_rgb;  /* dL/dC, or |dL/dC| for the mass */
    double gate_rel;      /* mass only */
} bwd_ctx;

/* Gradient of the rendered colour for a given dL/dC (grad_rgb[3R]).
 *
 * With C = sum_k w_k c_k + T_n bg, w_k = T_k (1 - exp(-sigma_k delta_k)),
 * T_{k+1} = T_k exp(-sigma_k delta_k) and R_k = sum_{j>k} w_j c_j + T_n bg
 * (everything the ray collects after sample k):
 *   dC/dsigma_k = delta_k (T_{k+1} c_k - R_k),
 *   dC/dc_k     = w_k.
 * Through the ReLUs (derivative 0 at 0), the SH basis and the trilinear
 * weights this gives the gradient of every corner value.  Gradients are
 * ADDED into grad_density[M] and grad_sh[M*27]; touched[M] is set to 1 for
 * every non-NULL corner of every sample of every ray (the active set). */
static void bwd_ray(const void *vctx, int64_t r, sparse_acc *acc)
{
    const bwd_ctx *cx = (const bwd_ctx *)vctx;
    const float *o = cx->rays_o + 3 * r, *d = cx->rays_d + 3 * r;
    int n = count_samples(cx->reso, cx->scale, cx->offset, cx->step, o, d);
    if (n == 0) return;
    sample_rec *recs = (sample_rec *)malloc(sizeof(sample_rec) * (size_t)n);
    double rgb[3], tau, T_n;
    const double *bgr = cx->bg + cx->bg_stride * r;
    march_ray(cx->reso, cx->scale, cx->offset, cx->step, cx->index, cx->density, cx->sh, o, d, bgr,
              recs, n, rgb, &tau, &T_n);
    double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
    double ylm[9];
    orc_sh_basis(dd, ylm);
    const double *g = cx->g_rgb + 3 * r;

    /* R = what the ray collects after the current sample, built from the
     * back so that it is a plain sum. */
    double R[3] = {T_n * bgr[0], T_n * bgr[1], T_n * bgr[2]};
    for (int k = n - 1; k >= 0; --k) {
        const sample_rec *s = &recs[k];
        double gc = 0.0, gR = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            gc += g[ch] * s->rgb[ch];
            gR += g[ch] * R[ch];
        }
        double dsig = s->sigma_pre > 0.0
                          ? s->delta * (s->T_next * gc - gR)
                          : 0.0;
        double dk[ORC_NSH];
        for (int ch = 0; ch < 3; ++ch) {
            double dcol = s->rgb_pre[ch] > 0.0 ? s->weight * g[ch] : 0.0;
            for (int l = 0; l < 9; ++l) dk[ch * 9 + l] = dcol * ylm[l];
        }
        for (int c = 0; c < 8; ++c) {
            int64_t id = s->ids[c];
            if (id < 0) continue;
            double wc = s->w[c];
            double *row = acc_row(acc, id);
            row[ORC_NSH] += wc * dsig;
            for (int q = 0; q < ORC_NSH; ++q) row[q] += wc * dk[q];
        }
        for (int ch = 0; ch < 3; ++ch) R[ch] += s->weight * s->rgb[ch];
    }
    free(recs);
}

void orc_render_bwd(const int32_t reso[3], const float scale[3],
                    const float offset[3], float step, const int32_t *index,
                    const double *density, const double *sh,
                    const float *rays_o, const float *rays_d, int64_t n_rays,
                    const double *bg, int64_t bg_stride, const double *grad_rgb,
                    double *grad_density, double *grad_sh, uint8_t *touched)
{
    bwd_ctx cx = {reso, scale, offset, step, index, density, sh, rays_o, rays_d, bg, bg_stride,
                  grad_rgb, 0.0};
    int64_t n_vox = 0;
    for (int64_t v = 0; v < (int64_t)reso[0] * reso[1] * reso[2]; ++v)
        if (index[v] >= n_vox) n_vox = index[v] + 1;
    accumulate_over_rays(n_rays, n_vox, bwd_ray, &cx, grad_density, grad_sh, touched);
}

/* Conditioning of the gradient sums, for tolerances: the same walk as
 * orc_render_bwd, but every term is ADDED in absolute value, with |dL/dC|
 * given in gabs_rgb[3R] (non-negative).  For sigma the term
 * delta (T_{k+1} g.c - g.R) contributes delta (T_{k+1} |g|.c + |g|.R), the
 * size of the two parts whose difference it is; for SH, |w_k g_ch Y_l|.
 * A float32 evaluation of the gradient can differ from the exact one by a
 * small multiple of the float32 unit roundoff times these sums.
 *
 * A ReLU gate (sigma_pre > 0, colour_pre > 0) is a discrete decision taken
 * from a rounded value: when |pre| <= gate_rel times the sum of the absolute
 * terms that form it, float32 may decide it either way, and both gradients
 * are correct.  Such terms enter the mass whether or not the gate is open
 * here, so the tolerance admits either decision. */
static void mass_ray(const void *vctx, int64_t r, sparse_acc *acc)
{
    const bwd_ctx *cx = (const bwd_ctx *)vctx;
    const double *density = cx->density, *sh = cx->sh;
    const double gate_rel = cx->gate_rel;
    const float *o = cx->rays_o + 3 * r, *d = cx->rays_d + 3 * r;
    int n = count_samples(cx->reso, cx->scale, cx->offset, cx->step, o, d);
    if (n == 0) return;
    sample_rec *recs = (sample_rec *)malloc(sizeof(sample_rec) * (size_t)n);
    double rgb[3], tau, T_n;
    const double *bgr = cx->bg + cx->bg_stride * r;
    march_ray(cx->reso, cx->scale, cx->offset, cx->step, cx->index, density, sh, o, d, bgr,
              recs, n, rgb, &tau, &T_n);
    double dd[3] = {(double)d[0], (double)d[1], (double)d[2]};
    double ylm[9];
    orc_sh_basis(dd, ylm);
    const double *g = cx->g_rgb + 3 * r;
    double R[3] = {T_n * fabs(bgr[0]), T_n * fabs(bgr[1]), T_n * fabs(bgr[2])};
    for (int k = n - 1; k >= 0; --k) {
        const sample_rec *s = &recs[k];
        /* absolute sums behind sigma_pre and the three colours */
        double abs_sig = 0.0, abs_col[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 8; ++c) {
            int64_t id = s->ids[c];
            if (id < 0) continue;
            abs_sig += s->w[c] * fabs(density[id]);
            for (int ch = 0; ch < 3; ++ch)
                for (int l = 0; l < 9; ++l)
                    abs_col[ch] += s->w[c] * fabs(sh[id * ORC_NSH + ch * 9 + l] * ylm[l]);
        }
        double gc = 0.0, gR = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            gc += g[ch] * fabs(s->rgb_pre[ch]);
            gR += g[ch] * R[ch];
        }
        int sig_on = s->sigma_pre > 0.0 || fabs(s->sigma_pre) <= gate_rel * abs_sig;
        double msig = sig_on ? s->delta * (s->T_next * gc + gR) : 0.0;
        double mk[ORC_NSH];
        for (int ch = 0; ch < 3; ++ch) {
            int on = s->rgb_pre[ch] > 0.0 || fabs(s->rgb_pre[ch]) <= gate_rel * abs_col[ch];
            double dcol = on ? s->weight * g[ch] : 0.0;
            for (int l = 0; l < 9; ++l) mk[ch * 9 + l] = dcol * fabs(ylm[l]);
        }
        for (int c = 0; c < 8; ++c) {
            int64_t id = s->ids[c];
            if (id < 0) continue;
            double wc = s->w[c];
            double *row = acc_row(acc, id);
            row[ORC_NSH] += wc * msig;
            for (int q = 0; q < ORC_NSH; ++q) row[q] += wc * mk[q];
        }
        for (int ch = 0; ch < 3; ++ch) R[ch] += s->weight * s->rgb[ch];
    }
    free(recs);
}

void orc_render_bwd_mass(const int32_t reso[3], const float scale[3],
                         const float offset[3], float step,
                         const int32_t *index, const double *density,
                         const double *sh, const float *rays_o,
                         const float *rays_d, int64_t n_rays,
                         const double *bg, int64_t bg_stride, const double *gabs_rgb,
                         double gate_rel, double *mass_density, double *mass_sh)
{
    bwd_ctx cx = {reso, scale, offset, step, index, density, sh, rays_o, rays_d, bg, bg_stride,
                  gabs_rgb, gate_rel};
    int64_t n_vox = 0;
    for (int64_t v = 0; v < (int64_t)reso[0] * reso[1] * reso[2]; ++v)
        if (index[v] >= n_vox) n_vox = index[v] + 1;
    accumulate_over_rays(n_rays, n_vox, mass_ray, &cx, mass_density, mass_sh, NULL);
}

/* ------------------------------------------------------------------------ */
/* The two optional priors of Sec. 3.7, on the rays of a batch:
 *   sparsity (Cauchy loss, after SNeRG):
 *     L_s = lambda_s sum_{rays, samples} log(1 + 2 sigma_k^2),
 *     sigma_k = the sample's density after the ReLU (the paper's "opacity"
 *     of the sample; reading of the design notes);
 *   beta prior on the foreground transmittance T = T_final of each ray
 *   (after Neural Volumes):
 *     L_b = lambda_b sum_rays [log(eps + T) + log(eps + 1 - T)],
 *     eps > 0 keeps the loss finite at T = 0 and T = 1 (the paper gives
 *     none; reading of the design notes), 1 - T = -expm1(-tau).
 * loss_out[0] += L_s, loss_out[1] += L_b.  Only densities enter either term:
 *   dL_s/dsigma_k = lambda_s 4 sigma_k / (1 + 2 sigma_k^2),
 *   dL_b/dsigma_k = dL_b/dT dT/dsigma_k = -delta_k T lambda_b
 *                   [1/(eps + T) - 1/(eps + 1 - T)]
 * (T = exp(-sum sigma delta)); both behind the density ReLU (derivative 0
 * at 0) and spread over the 8 corners by the trilinear weights into
 * grad_density[M] (ADDED; may be NULL).  mass_density[M] (ADDED; may be NULL)
 * gets the same sums in absolute value, with terms whose gate is ambiguous
 * (|sigma_pre| <= gate_rel times the sum of the absolute terms forming it)
 * counted whether or not the gate is open, as in orc_render_bwd_mass. */
void orc_regularisers(const int32_t reso[3], const float scale[3],
                      const float offset[3], float step, const int32_t *index,
                      const double *density, const double *sh,
                      const float *rays_o, const float *rays_d, int64_t n_rays,
                      double lambda_s, double lambda_b, double eps,
                      double gate_rel, double loss_out[2],
                      double *grad_density, double *mass_density)
{
    const double no_bg[3] = {0.0, 0.0, 0.0};
    double ls = 0.0, lb = 0.0;
    for (int64_t r = 0; r < n_rays; ++r) {
        const float *o = rays_o + 3 * r, *d = rays_d + 3 * r;
        int n = count_samples(reso, scale, offset, step, o, d);
        sample_rec *recs = n ? (sample_rec *)malloc((size_t)n * sizeof(sample_rec)) : NULL;
        double rgb[3], tau, T;
        march_ray(reso, scale, offset, step, index, density, sh, o, d, no_bg,
                  recs, n, rgb, &tau, &T);
        double one_minus_T = -expm1(-tau);
        lb += lambda_b * (log(eps + T) + log(eps + one_minus_T));
        double dLdT = lambda_b * (1.0 / (eps + T) - 1.0 / (eps + one_minus_T));
        for (int k = 0; k < n; ++k) {
            const sample_rec *s = &recs[k];
            double sig = s->sigma;
            ls += lambda_s * log1p(2.0 * sig * sig);
            double abs_sig = 0.0;
            for (int c = 0; c < 8; ++c)
                if (s->ids[c] >= 0) abs_sig += s->w[c] * fabs(density[s->ids[c]]);
            int open = s->sigma_pre > 0.0;
            int maybe = open || fabs(s->sigma_pre) <= gate_rel * abs_sig;
            double t_s = lambda_s * 4.0 * sig / (1.0 + 2.0 * sig * sig);
            double t_b = -s->delta * T * dLdT;
            for (int c = 0; c < 8; ++c) {
                int64_t id = s->ids[c];
                if (id < 0) continue;
                if (grad_density && open) grad_density[id] += s->w[c] * (t_s + t_b);
                if (mass_density && maybe) {
                    /* at an ambiguous gate the density may be rounded either
                     * side of 0: the Cauchy term is then at most the one at
                     * |sigma_pre| */
                    double a = fabs(s->sigma_pre);
                    double t_s_max = lambda_s * 4.0 * a / (1.0 + 2.0 * a * a);
                    mass_density[id] += s->w[c] * (fabs(t_s) + t_s_max + fabs(t_b));
                }
            }
        }
        free(recs);
    }
    loss_out[0] += ls;
    loss_out[1] += lb;
}

/* ------------------------------------------------------------------------ */
/* Total variation over the cells start, start+1, ..., start+count-1 (mod the
 * number of cells) in storage order (supplement B.1: contiguous segments of
 * the pointer grid).  For cell v and channel d:
 *   Delta_a = (D_a/256) (V_d(v + e_a) - V_d(v)),
 *   term    = sqrt(Delta_x^2 + Delta_y^2 + Delta_z^2 + eps).
 * sigma: NULL or out-of-range neighbours read 0.  SH: a NULL current cell has
 * no SH terms, and a NULL or out-of-range neighbour counts as equal to the
 * current cell (Delta = 0).  Loss = lambda_sigma/|V| sum term_sigma +
 * lambda_sh/|V| sum term_sh with |V| = count.  Gradients are ADDED; every
 * non-NULL voxel among v and its three forward neighbours is marked touched.
 * Returns the loss. */
static double tv_impl(const int32_t reso[3], const int32_t *index,
                      const double *density, const double *sh, int64_t start,
                      int64_t count, double lambda_sigma, double lambda_sh, double eps,
                      double *grad_density, double *grad_sh, uint8_t *touched,
                      int q_lo, int q_hi, int wrap_last)
{
    const int64_t ncell = (int64_t)reso[0] * reso[1] * reso[2];
    double s_axis[3];
    for (int a = 0; a < 3; ++a) s_axis[a] = (double)reso[a] / 256.0;
    const double inv_v = 1.0 / (double)count;
    double sum_sigma = 0.0, sum_sh = 0.0;

    for (int64_t c = 0; c < count; ++c) {
        int64_t v = ((start + c) % ncell + ncell) % ncell;
        int i = (int)(v / ((int64_t)reso[1] * reso[2]));
        int j = (int)((v / reso[2]) % reso[1]);
        int k = (int)(v % reso[2]);
        int64_t id = index[v];
        int64_t nid[3];
        int in_range[3] = {i + 1 < reso[0], j + 1 < reso[1], wrap_last || k + 1 < reso[2]};
        nid[0] = in_range[0] ? index[lin_id(reso, i + 1, j, k)] : -1;
        nid[1] = in_range[1] ? index[lin_id(reso, i, j + 1, k)] : -1;
        nid[2] = in_range[2] ? index[lin_id(reso, i, j, (k + 1) % reso[2])] : -1;

        /* density channel */
        {
            double x0 = id >= 0 ? density[id] : 0.0;
            double dlt[3], ss = 0.0;
            for (int a = 0; a < 3; ++a) {
                double xa = nid[a] >= 0 ? density[nid[a]] : 0.0;
                dlt[a] = s_axis[a] * (xa - x0);
                ss += dlt[a] * dlt[a];
            }
            double term = sqrt(ss + eps);
            sum_sigma += term;
            double scale = lambda_sigma * inv_v / term;
            if (id >= 0) {
                double gsum = 0.0;
                for (int a = 0; a < 3; ++a) gsum += s_axis[a] * dlt[a];
                grad_density[id] -= scale * gsum;
                touched[id] = 1;
            }
            for (int a = 0; a < 3; ++a) {
                if (nid[a] < 0) continue;
                grad_density[nid[a]] += scale * s_axis[a] * dlt[a];
                touched[nid[a]] = 1;
            }
        }
        /* SH channels */
        if (id >= 0) {
            for (int q = q_lo; q < q_hi; ++q) {
                double x0 = sh[id * ORC_NSH + q];
                double dlt[3], ss = 0.0;
                for (int a = 0; a < 3; ++a) {
                    dlt[a] = nid[a] >= 0
                                 ? s_axis[a] * (sh[nid[a] * ORC_NSH + q] - x0)
                                 : 0.0;
                    ss += dlt[a] * dlt[a];
                }
                double term = sqrt(ss + eps);
                sum_sh += term;
                double scale = lambda_sh * inv_v / term;
                double gsum = 0.0;
                for (int a = 0; a < 3; ++a) {
                    if (nid[a] < 0) continue;
                    gsum += s_axis[a] * dlt[a];
                    grad_sh[nid[a] * ORC_NSH + q] += scale * s_axis[a] * dlt[a];
                }
                grad_sh[id * ORC_NSH + q] -= scale * gsum;
            }
        }
    }
    return lambda_sigma * inv_v * sum_sigma + lambda_sh * inv_v * sum_sh;
}

double orc_tv(const int32_t reso[3], const int32_t *index,
              const double *density, const double *sh, int64_t start,
              int64_t count, double lambda_sigma, double lambda_sh, double eps,
              double *grad_density, double *grad_sh, uint8_t *touched)
{
    return tv_impl(reso, index, density, sh, start, count, lambda_sigma, lambda_sh, eps,
                   grad_density, grad_sh, touched, 0, ORC_NSH, 0);
}

/* The same TV on an MSI background grid (reso (L, H, W)): the colour terms
 * are its three colour coefficients (sh slots 24-26) instead of the 27 SH
 * coefficients, and the azimuth axis (the last) wraps around: the
 * neighbour of column W-1 is column 0 (supplement B.1: the background's TV
 * wraps around the edges of the equirectangular image). */
double orc_bg_tv(const int32_t reso[3], const int32_t *index,
                 const double *density, const double *sh, int64_t start,
                 int64_t count, double lambda_sigma, double lambda_color, double eps,
                 double *grad_density, double *grad_sh, uint8_t *touched)
{
    return tv_impl(reso, index, density, sh, start, count, lambda_sigma, lambda_color, eps,
                   grad_density, grad_sh, touched, ORC_BG_SLOT, ORC_BG_SLOT + 3, 1);
}

/* ------------------------------------------------------------------------ */
/* RMSProp (Sec. 3.5) on the active voxels only: for each of the 28 values of
 * an active voxel, v <- beta v + (1-beta) g^2, p <- p - lr g / (sqrt(v) + eps),
 * then the gradient is cleared.  lr_sigma for density, lr_sh for SH.
 * Inactive voxels (parameters, state and gradient) are left as they are. */
void orc_rmsprop(int64_t n_vox, const uint8_t *active, double *density,
                 double *sh, double *v_density, double *v_sh,
                 double *grad_density, double *grad_sh, double lr_sigma,
                 double lr_sh, double beta, double eps)
{
    for (int64_t m = 0; m < n_vox; ++m) {
        if (!active[m]) continue;
        {
            double g = grad_density[m];
            v_density[m] = beta * v_density[m] + (1.0 - beta) * g * g;
            density[m] -= lr_sigma * g / (sqrt(v_density[m]) + eps);
            grad_density[m] = 0.0;
        }
        for (int q = 0; q < ORC_NSH; ++q) {
            int64_t p = m * ORC_NSH + q;
            double g = grad_sh[p];
            v_sh[p] = beta * v_sh[p] + (1.0 - beta) * g * g;
            sh[p] -= lr_sh * g / (sqrt(v_sh[p]) + eps);
            grad_sh[p] = 0.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Grid creation: table ids in increasing storage order of the occupied
 * cells.  Returns the number of occupied cells. */
int64_t orc_grid_create(const int32_t reso[3], const uint8_t *mask,
                        int32_t *index_out)
{
    const int64_t ncell = (int64_t)reso[0] * reso[1] * reso[2];
    int64_t m = 0;
    for (int64_t v = 0; v < ncell; ++v) index_out[v] = mask[v] ? (int32_t)m++ : -1;
    return m;
}

/* Largest sample weight seen by each voxel, the statistic of pruning by
 * weight (Sec. 3.4, the method taken from PlenOctrees; supplement B.1 for
 * the thresholds).  The weight of sample k is its compositing weight in
 * Eq. (1), w_k = T_k (1 - exp(-sigma_k delta_k)).  A voxel's statistic is
 * the largest w_k over the samples whose trilinear interpolation reads it,
 * i.e. the samples whose cell has it as one of its 8 corners.  wmax[M] is
 * raised in place (wmax[id] = max(wmax[id], w_k)), so calls over batches of
 * rays give the maximum over all of them. */
void orc_max_weight(const int32_t reso[3], const float scale[3],
                    const float offset[3], float step, const int32_t *index,
                    const double *density, const double *sh,
                    const float *rays_o, const float *rays_d, int64_t n_rays,
                    double *wmax)
{
    const double no_bg[3] = {0.0, 0.0, 0.0};
    for (int64_t r = 0; r < n_rays; ++r) {
        const float *o = rays_o + 3 * r, *d = rays_d + 3 * r;
        int n = count_samples(reso, scale, offset, step, o, d);
        if (n == 0) continue;
        sample_rec *recs = (sample_rec *)malloc((size_t)n * sizeof(sample_rec));
        double rgb[3], tau, tf;
        march_ray(reso, scale, offset, step, index, density, sh, o, d, no_bg,
                  recs, n, rgb, &tau, &tf);
        for (int k = 0; k < n; ++k)
            for (int c = 0; c < 8; ++c) {
                int64_t id = recs[k].ids[c];
                if (id >= 0 && recs[k].weight > wmax[id]) wmax[id] = recs[k].weight;
            }
        free(recs);
    }
}

/* Threshold pruning with dilation (Sec. 3.4; supplement B.1 for the
 * thresholds).  value[M] is the per-voxel statistic: the stored density for
 * pruning by density, the maximum sample weight (orc_max_weight) for pruning
 * by weight.  A voxel counts as occupied when it is non-NULL and its value is
 * >= thresh.  A non-NULL voxel is kept when it or any of its 26 neighbours
 * is occupied.  keep_out[ncell] gets 1 for kept voxels.  Returns the number
 * kept; *n_pruned gets the number of non-NULL voxels removed. */
int64_t orc_prune_mask(const int32_t reso[3], const int32_t *index,
                       const double *value, double thresh, uint8_t *keep_out,
                       int64_t *n_pruned)
{
    int64_t kept = 0, pruned = 0;
    for (int i = 0; i < reso[0]; ++i)
        for (int j = 0; j < reso[1]; ++j)
            for (int k = 0; k < reso[2]; ++k) {
                int64_t v = lin_id(reso, i, j, k);
                keep_out[v] = 0;
                if (index[v] < 0) continue;
                int any = 0;
                for (int a = -1; a <= 1 && !any; ++a)
                    for (int b = -1; b <= 1 && !any; ++b)
                        for (int c = -1; c <= 1 && !any; ++c) {
                            int ii = i + a, jj = j + b, kk = k + c;
                            if (ii < 0 || jj < 0 || kk < 0 || ii >= reso[0] ||
                                jj >= reso[1] || kk >= reso[2])
                                continue;
                            int32_t id = index[lin_id(reso, ii, jj, kk)];
                            if (id >= 0 && value[id] >= thresh) any = 1;
                        }
                if (any) {
                    keep_out[v] = 1;
                    ++kept;
                } else {
                    ++pruned;
                }
            }
    *n_pruned = pruned;
    return kept;
}

/* Resampling to a new resolution (Sec. 3.4: trilinear initialisation after
 * subdivision, arbitrary ratios allowed).  New voxel j along an axis is
 * occupied when its parent cell p = floor((2j+1) N_old / (2 N_new)) is
 * occupied.  Its values are the trilinear interpolation of the old field
 * (NULL = 0) at old grid coordinate ((j + 0.5) N_old / N_new) - 0.5, clamped
 * to [0, N_old - 1].  Writes index_new (new table in storage order) and the
 * new density/SH (sized by the caller from orc_upsample_count).  Returns the
 * new voxel count. */
int64_t orc_upsample_count(const int32_t reso[3], const int32_t *index,
                           const int32_t new_reso[3])
{
    int64_t m = 0;
    for (int i = 0; i < new_reso[0]; ++i) {
        int pi = (int)(((int64_t)(2 * i + 1) * reso[0]) / (2 * (int64_t)new_reso[0]));
        for (int j = 0; j < new_reso[1]; ++j) {
            int pj = (int)(((int64_t)(2 * j + 1) * reso[1]) / (2 * (int64_t)new_reso[1]));
            for (int k = 0; k < new_reso[2]; ++k) {
                int pk = (int)(((int64_t)(2 * k + 1) * reso[2]) / (2 * (int64_t)new_reso[2]));
                if (index[lin_id(reso, pi, pj, pk)] >= 0) ++m;
            }
        }
    }
    return m;
}

static void upsample_coord(int j, int n_old, int n_new, int *i0, double *f)
{
    double g = ((double)j + 0.5) * (double)n_old / (double)n_new - 0.5;
    if (g < 0.0) g = 0.0;
    if (g > (double)(n_old - 1)) g = (double)(n_old - 1);
    int c = (int)floor(g);
    if (c > n_old - 2) c = n_old - 2;
    if (c < 0) c = 0;
    *i0 = c;
    *f = g - (double)c;
}

int64_t orc_upsample(const int32_t reso[3], const int32_t *index,
                     const double *density, const double *sh,
                     const int32_t new_reso[3], int32_t *index_new,
                     double *density_new, double *sh_new)
{
    int64_t m = 0;
    for (int i = 0; i < new_reso[0]; ++i) {
        int pi = (int)(((int64_t)(2 * i + 1) * reso[0]) / (2 * (int64_t)new_reso[0]));
        for (int j = 0; j < new_reso[1]; ++j) {
            int pj = (int)(((int64_t)(2 * j + 1) * reso[1]) / (2 * (int64_t)new_reso[1]));
            for (int k = 0; k < new_reso[2]; ++k) {
                int pk = (int)(((int64_t)(2 * k + 1) * reso[2]) / (2 * (int64_t)new_reso[2]));
                int64_t v = lin_id(new_reso, i, j, k);
                if (index[lin_id(reso, pi, pj, pk)] < 0) {
                    index_new[v] = -1;
                    continue;
                }
                index_new[v] = (int32_t)m;
                int cell[3];
                double f[3];
                upsample_coord(i, reso[0], new_reso[0], &cell[0], &f[0]);
                upsample_coord(j, reso[1], new_reso[1], &cell[1], &f[1]);
                upsample_coord(k, reso[2], new_reso[2], &cell[2], &f[2]);
                double sig, kc[ORC_NSH], w[8];
                int64_t ids[8];
                interpolate(reso, index, density, sh, cell, f, &sig, kc, ids, w);
                density_new[m] = sig;
                for (int q = 0; q < ORC_NSH; ++q) sh_new[m * ORC_NSH + q] = kc[q];
                ++m;
            }
        }
    }
    return m;
}

/* Learning-rate schedules (supplement B.1).  Log-linear decay from lr0 at
 * step 0 to lr1 at step max_steps; with delay_steps > 0 it is scaled by
 * mult + (1 - mult) sin(pi/2 min(1, step/delay_steps)) (the delayed form of
 * the JAXNeRF / Mip-NeRF schedule). */
double orc_lr_schedule(double step, double lr0, double lr1, double max_steps,
                       double delay_steps, double delay_mult)
{
    const double pi = 3.14159265358979323846;
    double frac = step / max_steps;
    if (frac > 1.0) frac = 1.0;
    double lr = exp((1.0 - frac) * log(lr0) + frac * log(lr1));
    if (delay_steps > 0.0) {
        double u = step / delay_steps;
        if (u > 1.0) u = 1.0;
        lr *= delay_mult + (1.0 - delay_mult) * sin(0.5 * pi * u);
    }
    return lr;
}
