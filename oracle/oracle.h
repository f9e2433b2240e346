/*
 * FP64 reference ("oracle") for the ray-cast colouring and filtering path of
 * Vohl, Fluke, Barnes & Hassan (2017), "Real-time colouring and filtering with
 * graphics shaders".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header or constant
 * with the HIP library and is deliberately plain and slow: one ray at a time, no
 * bricking, no fusion, every step in double precision in the order the paper gives.
 *
 * Cube layout: C-order [z][y][x], x fastest (x = RA, y = Dec, z = velocity).
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Appendix A: parallel (type 0) or perspective (type 1) projection. */
typedef struct {
    int32_t type;
    double eye[3], U[3], V[3], W[3];
    int32_t width, height;
} orc_camera;

/* Transfer functions of Section 3 (Alg. MIP0, AVIP0, MIP1, AVIP1, MIP_RGB, AVIP_RGB). */
enum { ORC_MIP0 = 0, ORC_MIP1 = 1, ORC_MIPRGB = 2, ORC_AVIP0 = 3, ORC_AVIP1 = 4, ORC_AVIPRGB = 5 };
/* Section 4 filters: none, intensity clipping, intensity domain scaling. */
enum { ORC_FILTER_NONE = 0, ORC_FILTER_CLIP = 1, ORC_FILTER_SCALE = 2 };

typedef struct {
    int32_t mode;             /* ORC_MIP0 .. ORC_AVIPRGB */
    int32_t filter;           /* ORC_FILTER_* */
    int32_t box_arm;          /* Section 4.1 filterArm (0 = no box smoothing) */
    int32_t mip_alpha;        /* 0: table alpha / s_max, 1: opaque, 2: transparent only at or below minT */
    int32_t ratio;            /* 0 none, 1 line ratio method 1, 2 method 2 (Section 4.5) */
    int32_t opacity_from_lut; /* 0: a = k*s (Alg. AVIP0); 1: a = k*table(s).a */
    double k, min_val, ert;   /* AVIP weighting factor, minVal, termination threshold (0.99) */
    double lo, hi;            /* colour-map domain; DATAMIN = lo */
    double dt;                /* step along the unit ray direction, in voxels */
    double min_t, max_t;      /* thresholds (cube 1 for the ratio methods) */
    double min_t2, max_t2;    /* thresholds for cube 2 (ratio methods) */
    double ratio_lo, ratio_hi;/* domain the ratio is normalised over */
    /* In-ray 3-axis Gaussian of Section 4.2 (Alg. 9-tap smoothing), star_n > 0 to enable:
     * the one-axis stencil c0 v + sum_k w_k (cube[p + off_k e] + cube[p - off_k e]) applied
     * along x, then y, then z, each axis taking the previous result as its centre value.
     * PARITY UNPINNED in general (how the paper combines the three axes is a reading); the
     * one-axis reductions are pinned. */
    int32_t star_n;           /* number of (off, w) pairs, 0..4 */
    double star_c0;
    double star_off[4], star_w[4];
} orc_params;

/* Margins below which a discrete decision counts as "could flip" (fragile pixel). */
typedef struct {
    double ds;  /* MIP argmax: gap between the maximum and another sample (s units) */
    double dv;  /* threshold tests on raw values: |v - threshold| */
    double da;  /* early termination: |alpha - ert| */
    double dn;  /* sample count: distance of L/dt from an integer, relative */
    double dr;  /* ratio denominators: |v1| below this makes the ratio ill-conditioned */
    double pv;  /* conditioning probe: every sampled value is moved by +pv (all samples),
                   by +-pv (pseudo-random signs), by a ramp from -pv to +pv along the ray,
                   and for two cubes by +pv on the first and -pv on the second; 0 disables
                   the probe */
    double pt;  /* ... and the pixel is fragile when its RGBA then moves by more than pt */
    double pp;  /* ... and every sample position coordinate x by +-pp (|x| + 1) (relative
                   rounding scale of a float32 position) */
} orc_margins;

/* Fragility bits reported per pixel (0 = robust). */
enum {
    ORC_FRAG_COUNT = 1,      /* (t1 - t0)/dt within dn of an integer: N could differ by one */
    ORC_FRAG_ARGMAX = 2,     /* MIP1/MIP_RGB: another sample within ds of the maximum */
    ORC_FRAG_ERT = 4,        /* AVIP: alpha within da of the termination threshold */
    ORC_FRAG_THRESHOLD = 8,  /* a filtered value within dv of minT/maxT (or of 0 for ratios) */
    ORC_FRAG_RATIO = 16,     /* ratio denominator below dr */
    ORC_FRAG_COND = 32,      /* the +-pv / +-pp probe moved the RGBA by more than pt */
    ORC_NOT_CANDIDATE = 64   /* forced arg-max: the forced sample is not within ds of the
                                maximum (so it is not a valid arg-max) */
};

/* Render npix pixels (pix == NULL: all width*height pixels, row-major).  V2 is the second
 * cube for the ratio methods (NULL otherwise).  lut: M RGBA entries at j/(M-1).
 * Outputs rgba[4*npix], fragile[npix] (ORC_FRAG_* bits), nsamples[npix] (may be NULL).
 * forced_n (may be NULL): per pixel, when >= 0 an AVIP ray composites exactly that many
 * samples instead of stopping at the threshold (the other reading of a near-threshold
 * termination), and a MIP1 / MIP_RGB ray takes sample forced_n as its arg-max (the other
 * reading of a near tie of the maximum; ORC_NOT_CANDIDATE flags a sample further than ds
 * below the maximum, or past the ray's end).  Returns 0 on success, nonzero on invalid
 * arguments. */
int orc_render(const double* V, const double* V2, int32_t nx, int32_t ny, int32_t nz,
               const orc_camera* cam, const double* lut, int32_t M, const orc_params* p,
               const orc_margins* mg, int64_t npix, const int64_t* pix,
               const int32_t* forced_n, double* rgba, uint8_t* fragile, int32_t* nsamples,
               int32_t nthreads);

/* Ray of pixel (px, py): origin o and unit direction d.  Entry/exit of the cell-centred
 * box [-0.5, n-0.5]^3.  Returns 1 and t0 < t1 when the ray (t >= 0) meets the box. */
void orc_pixel_ray(const orc_camera* cam, int32_t px, int32_t py, double o[3], double d[3]);
int orc_ray_box(int32_t nx, int32_t ny, int32_t nz, const double o[3], const double d[3],
                double* t0, double* t1);
/* Trilinear sample with clamp-to-edge at point p (voxel centres at integers). */
double orc_trilinear(const double* V, int32_t nx, int32_t ny, int32_t nz, const double p[3]);

/* AVIP0 with a piecewise-linear RGBA transfer function (colour = tf(s).rgb, opacity =
 * k * tf(s).a), and its reverse-mode derivative, storing every sample.  grad_rgba holds
 * dL/dRGBA for the npix pixels; grad_tf[M*4] and grad_vox[nx*ny*nz] are ACCUMULATED
 * (caller zeroes them).  Single-threaded, deterministic. */
int orc_render_grad(const double* V, int32_t nx, int32_t ny, int32_t nz,
                    const orc_camera* cam, const double* tf, int32_t M, const orc_params* p,
                    int64_t npix, const int64_t* pix, const double* grad_rgba,
                    double* rgba, double* grad_tf, double* grad_vox);

/* Separable 3D smoothing with clamp-to-edge: out = (g x g x g) applied along x, then y,
 * then z.  taps g[0..T-1], T odd, centred.  tmp: scratch of nx*ny*nz doubles. */
int orc_smooth(const double* V, int32_t nx, int32_t ny, int32_t nz, const double* g,
               int32_t T, double* out, double* tmp, int32_t nthreads);
/* Same operator evaluated at selected voxels by the direct triple sum. */
int orc_smooth_at(const double* V, int32_t nx, int32_t ny, int32_t nz, const double* g,
                  int32_t T, int64_t npts, const int64_t* idx, double* out);

/* Voxel-wise line ratio of two equal-length spectral windows of one cube. */
int orc_line_ratio(const double* V, int32_t nx, int32_t ny, int32_t nz, int32_t z0a,
                   int32_t z0b, int32_t nzw, double min_t_a, double min_t_b, double datamin,
                   double* out);

/* Moment maps of every spectrum over channels [z0, z0 + nzw) (Section 2.2, Eq. mom0 and
 * Eq. mom1, and the argmax variant).  A channel counts when its value is finite and inside
 * [min_t, max_t].  m0 = dv * sum v; m1 = sum z v / sum v with z the cube's channel index (NaN
 * when no channel counts or the sum is zero); amax = the last channel holding the largest
 * counted value (-1 when none counts).  Outputs [ny][nx]. */
int orc_moments(const double* V, int32_t nx, int32_t ny, int32_t nz, int32_t z0, int32_t nzw,
                double dv, double min_t, double max_t, double* m0, double* m1, int32_t* amax);

#ifdef __cplusplus
}
#endif
#endif
