/*
 * FP64 reference ("oracle") -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Every function follows the paper's definitions step by step:
 *   Alg. 1 (outline of front-to-back ray tracing), Eq. MIP and Eq. AVIP (Section 2.2),
 *   Alg. MIP0 / AVIP0 (Section 3.1), MIP1 / AVIP1 (Section 3.2), MIP_RGB / AVIP_RGB
 *   (Section 3.3), box smoothing (Section 4.1), Gaussian / binomial smoothing (Section 4.2),
 *   intensity clipping and domain scaling (Sections 4.3, 4.4), line-ratio methods 1 and 2
 *   (Section 4.5), parallel/perspective projection (Appendix A).
 * Where the paper is silent the reading used is stated next to the code.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }
static double lerpd(double a, double b, double f) { return a + f * (b - a); }

/* Appendix A.  Pixel centre (px+0.5, py+0.5) maps to u, v in (-1, 1).  Parallel rays start
 * on the image plane eye + uU + vV and travel along W; perspective rays leave the eye
 * along W + uU + vV.  Directions are normalised so t counts voxels. */
void orc_pixel_ray(const orc_camera* c, int32_t px, int32_t py, double o[3], double d[3]) {
    double u = 2.0 * (px + 0.5) / c->width - 1.0;
    double v = 2.0 * (py + 0.5) / c->height - 1.0;
    for (int a = 0; a < 3; ++a) {
        if (c->type == 0) {
            o[a] = c->eye[a] + u * c->U[a] + v * c->V[a];
            d[a] = c->W[a];
        } else {
            o[a] = c->eye[a];
            d[a] = c->W[a] + u * c->U[a] + v * c->V[a];
        }
    }
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] = d[0] / len;
    d[1] = d[1] / len;
    d[2] = d[2] / len;
}

/* Reading: voxel (i, j, l) is centred at (i, j, l); the volume box is the cell-centred
 * [-0.5, n-0.5] on each axis (the texel-centre convention of a 3D texture).  Slab test;
 * the part of the ray behind its origin is cut off (eye inside the box). */
int orc_ray_box(int32_t nx, int32_t ny, int32_t nz, const double o[3], const double d[3],
                double* t0, double* t1) {
    const int32_t n[3] = {nx, ny, nz};
    double tn = -INFINITY, tf = INFINITY;
    if (!(isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]))) return 0;
    for (int a = 0; a < 3; ++a) {
        double lo = -0.5, hi = n[a] - 0.5;
        if (d[a] == 0.0) {
            if (o[a] < lo || o[a] > hi) return 0;
            continue;
        }
        double ta = (lo - o[a]) / d[a];
        double tb = (hi - o[a]) / d[a];
        if (ta > tb) { double t = ta; ta = tb; tb = t; }
        if (ta > tn) tn = ta;
        if (tb < tf) tf = tb;
    }
    if (tn < 0.0) tn = 0.0;
    if (!(tf > tn)) return 0;
    *t0 = tn;
    *t1 = tf;
    return 1;
}

/* The 3D-texture fetch cube[loc] of Alg. 1, as trilinear interpolation with
 * clamp-to-edge: each coordinate is clamped to [0, n-1], then interpolated along x, y, z. */
double orc_trilinear(const double* V, int32_t nx, int32_t ny, int32_t nz, const double p[3]) {
    double x = clampd(p[0], 0.0, nx - 1.0);
    double y = clampd(p[1], 0.0, ny - 1.0);
    double z = clampd(p[2], 0.0, nz - 1.0);
    int64_t i0 = (int64_t)floor(x), j0 = (int64_t)floor(y), l0 = (int64_t)floor(z);
    int64_t i1 = i0 + 1 < nx ? i0 + 1 : nx - 1;
    int64_t j1 = j0 + 1 < ny ? j0 + 1 : ny - 1;
    int64_t l1 = l0 + 1 < nz ? l0 + 1 : nz - 1;
    double fx = x - (double)i0, fy = y - (double)j0, fz = z - (double)l0;
#define AT(i, j, l) V[((l) * (int64_t)ny + (j)) * (int64_t)nx + (i)]
    double c00 = lerpd(AT(i0, j0, l0), AT(i1, j0, l0), fx);
    double c10 = lerpd(AT(i0, j1, l0), AT(i1, j1, l0), fx);
    double c01 = lerpd(AT(i0, j0, l1), AT(i1, j0, l1), fx);
    double c11 = lerpd(AT(i0, j1, l1), AT(i1, j1, l1), fx);
#undef AT
    double c0 = lerpd(c00, c10, fy);
    double c1 = lerpd(c01, c11, fy);
    return lerpd(c0, c1, fz);
}

/* colourMap(s): reading -- a table of M RGBA entries at s = j/(M-1), linearly
 * interpolated (a lookup table, Section 2.1). */
static void table_at(const double* L, int32_t M, double s, double out[4]) {
    double x = s * (M - 1);
    int64_t j0 = (int64_t)floor(x);
    if (j0 > M - 2) j0 = M - 2;
    if (j0 < 0) j0 = 0;
    double f = x - (double)j0;
    for (int ch = 0; ch < 4; ++ch) out[ch] = lerpd(L[4 * j0 + ch], L[4 * (j0 + 1) + ch], f);
}

/* Map a value onto the colour-map domain [lo, hi] -> [0, 1]. */
static double domain01(double v, double lo, double hi) {
    return hi > lo ? clampd((v - lo) / (hi - lo), 0.0, 1.0) : 0.0;
}

typedef struct {
    const double *V, *V2;
    int32_t nx, ny, nz;
    const double* lut;
    int32_t M;
    const orc_params* p;
    const orc_margins* mg;
    double o[3], d[3], t0;
    int64_t pix;     /* pixel id (seeds the conditioning probe) */
    int pert;        /* 0: exact values; 1..4: probe patterns */
    int64_t nsamp;   /* samples on this ray (the ramp pattern spans them) */
} ray_ctx;

/* Deterministic +-1 for the conditioning probe (splitmix64 finaliser of pixel, sample, cube). */
static double probe_sign(int64_t pix, int64_t k, int salt) {
    uint64_t z = (uint64_t)pix * 0x9E3779B97F4A7C15ull;
    z ^= (uint64_t)(k + 4099) * 0xBF58476D1CE4E5B9ull;
    z ^= (uint64_t)salt * 0x94D049BB133111EBull;
    z ^= z >> 31;
    z *= 0xD6E8FEB86659FD93ull;
    z ^= z >> 32;
    return (z & 1u) ? 1.0 : -1.0;
}

static void ray_point(const ray_ctx* r, int64_t k, double q[3]) {
    double t = r->t0 + (double)k * r->p->dt;
    for (int a = 0; a < 3; ++a) q[a] = r->o[a] + t * r->d[a];
}

/* loc of Alg. 1 in normalised texture coordinates: clamp((p + 0.5)/n, 0, 1). */
static void ray_loc(const ray_ctx* r, int64_t k, double loc[3]) {
    double q[3];
    ray_point(r, k, q);
    loc[0] = clampd((q[0] + 0.5) / r->nx, 0.0, 1.0);
    loc[1] = clampd((q[1] + 0.5) / r->ny, 0.0, 1.0);
    loc[2] = clampd((q[2] + 0.5) / r->nz, 0.0, 1.0);
}

/* Section 4.2's in-shader Gaussian at point q (Alg. 9-tap smoothing, applied to each data
 * axis in turn, x then y then z): smooth(oVal, direction) = oVal c0 + sum over the offset
 * pairs of w_k (cube[q + off_k e] + cube[q - off_k e]), in the printed order; the result of
 * one axis is the oVal of the next.  Every lookup is the trilinear fetch of the raw cube. */
static double star_sample(const ray_ctx* r, const double* V, const double q[3]) {
    const orc_params* p = r->p;
    double val = orc_trilinear(V, r->nx, r->ny, r->nz, q);
    for (int a = 0; a < 3; ++a) {
        double acc = 0.0;
        acc = acc + val * p->star_c0;
        for (int k = 0; k < p->star_n; ++k) {
            double qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
            qp[a] += p->star_off[k];
            qm[a] -= p->star_off[k];
            acc = acc + orc_trilinear(V, r->nx, r->ny, r->nz, qp) * p->star_w[k];
            acc = acc + orc_trilinear(V, r->nx, r->ny, r->nz, qm) * p->star_w[k];
        }
        val = acc;
    }
    return val;
}

/* cube[loc] followed by smooth() of Alg. 1: the box mean of the 2a+1 samples taken at the
 * ray's own positions k-a .. k+a (Section 4.1, "along the ray direction"), or the in-ray
 * Gaussian of Section 4.2. */
static double ray_sample(const ray_ctx* r, const double* V, int64_t k, int which) {
    double q[3];
    ray_point(r, k, q);
    if (r->pert && r->mg->pp > 0.0)
        for (int a = 0; a < 3; ++a)
            q[a] += r->mg->pp * (fabs(q[a]) + 1.0) * probe_sign(r->pix, k, 16 * r->pert + 4 + a);
    double v = r->p->star_n > 0 ? star_sample(r, V, q) : orc_trilinear(V, r->nx, r->ny, r->nz, q);
    if (r->pert == 1) v += r->mg->pv;  /* correlated error: every sample moved up */
    if (r->pert == 2) v += r->mg->pv * probe_sign(r->pix, k, 16 + which);  /* random signs */
    if (r->pert == 3) v += which ? -r->mg->pv : r->mg->pv;  /* the two cubes move apart */
    if (r->pert == 4) {  /* an error growing along the ray, as position rounding does */
        const double span = r->nsamp > 1 ? (double)(r->nsamp - 1) : 1.0;
        v += r->mg->pv * (2.0 * (double)k / span - 1.0);
    }
    return v;
}

static double ray_value(const ray_ctx* r, const double* V, int64_t k, int which) {
    int32_t arm = r->p->box_arm;
    if (arm <= 0) return ray_sample(r, V, k, which);
    double sum = 0.0;
    for (int64_t j = -arm; j <= arm; ++j) sum += ray_sample(r, V, k + j, which);
    return sum / (double)(2 * arm + 1);
}

/* filter() of Alg. 1 followed by the mapping onto [0, 1].
 *   none:  s = (v - lo)/(hi - lo) clamped.
 *   clip (Section 4.3): v < minT or v > maxT -> DATAMIN (= lo), then as none.
 *   scale (Section 4.4): v outside [minT, maxT] -> DATAMIN (s = 0), else
 *          s = (v - minT)/(maxT - minT).
 * *exact is set when s came from a discrete branch well away from its boundary (so any
 * correct implementation produces the identical s). */
static double filter_s(const orc_params* p, double v, double dv, int* fragile, int* exact) {
    *exact = 0;
    if (p->filter == ORC_FILTER_CLIP || p->filter == ORC_FILTER_SCALE) {
        if (fabs(v - p->min_t) < dv || fabs(v - p->max_t) < dv) *fragile |= ORC_FRAG_THRESHOLD;
        if (p->filter == ORC_FILTER_CLIP) {
            if (v < p->min_t) { v = p->lo; *exact = 1; }
            if (v > p->max_t) { v = p->lo; *exact = 1; }
            return domain01(v, p->lo, p->hi);
        }
        if (v > p->max_t || v < p->min_t) { *exact = 1; return 0.0; }
        return (v - p->min_t) / (p->max_t - p->min_t);
    }
    if (v <= p->lo - dv || v >= p->hi + dv) *exact = 1;
    return domain01(v, p->lo, p->hi);
}

/* Clip applied to one raw value for the ratio methods (Section 4.5 figures use
 * clipping on both cubes, each with its own minimum threshold). */
static double clip_raw(const orc_params* p, double v, double mn, double mx, double dv,
                       int* fragile) {
    if (p->filter != ORC_FILTER_CLIP) return v;
    if (fabs(v - mn) < dv || fabs(v - mx) < dv) *fragile |= ORC_FRAG_THRESHOLD;
    if (v < mn) v = p->lo;
    if (v > mx) v = p->lo;
    return v;
}

static void render_core(const ray_ctx* base, const orc_camera* cam, int32_t px, int32_t py,
                        int pert, int32_t forced, double out[4], uint8_t* frag_out,
                        int32_t* ns_out, double* sbuf, uint8_t* ebuf) {
    const orc_params* p = base->p;
    const orc_margins* mg = base->mg;
    ray_ctx r = *base;
    int fragile = 0;
    int64_t count = 0;
    double t1;
    r.pix = (int64_t)py * cam->width + px;
    r.pert = pert;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    *frag_out = 0;
    if (ns_out) *ns_out = 0;

    orc_pixel_ray(cam, px, py, r.o, r.d);
    if (!orc_ray_box(r.nx, r.ny, r.nz, r.o, r.d, &r.t0, &t1)) return; /* miss -> (0,0,0,0) */

    /* Reading: samples t_k = t0 + k dt, k = 0 .. N-1, N = ceil((t1 - t0)/dt). */
    double q = (t1 - r.t0) / p->dt;
    int64_t N = (int64_t)ceil(q);
    r.nsamp = N;
    {
        double near = fabs(q - nearbyint(q));
        if (near > 0.0 && near < mg->dn * (q > 1.0 ? q : 1.0)) fragile |= ORC_FRAG_COUNT;
    }

    if (p->ratio == 1) {
        /* Line ratio, method 1: MIP of each cube with strict '>', then colourMap(max2/max1)
         * when max1 > 0, else (0,0,0,0). */
        double m1 = -INFINITY, m2 = -INFINITY;
        for (int64_t k = 0; k < N; ++k) {
            double v1 = clip_raw(p, ray_value(&r, r.V, k, 0), p->min_t, p->max_t, mg->dv, &fragile);
            double v2 = clip_raw(p, ray_value(&r, r.V2, k, 1), p->min_t2, p->max_t2, mg->dv, &fragile);
            if (v1 > m1) m1 = v1;
            if (v2 > m2) m2 = v2;
        }
        count = N;
        if (fabs(m1) < mg->dv) fragile |= ORC_FRAG_THRESHOLD;
        if (m1 > 0.0) {
            if (m1 < mg->dr) fragile |= ORC_FRAG_RATIO;
            double s = domain01(m2 / m1, p->ratio_lo, p->ratio_hi);
            table_at(r.lut, r.M, s, out);
            if (p->mip_alpha == 1) out[3] = 1.0;
        }
    } else if (p->ratio == 2) {
        /* Line ratio, method 2: per-sample ratio cube2/cube1 when cube1 > 0, else DATAMIN
         * (s = 0); then MIP0. */
        double smax = -INFINITY;
        for (int64_t k = 0; k < N; ++k) {
            double v1 = clip_raw(p, ray_value(&r, r.V, k, 0), p->min_t, p->max_t, mg->dv, &fragile);
            double v2 = clip_raw(p, ray_value(&r, r.V2, k, 1), p->min_t2, p->max_t2, mg->dv, &fragile);
            double s;
            if (fabs(v1) < mg->dv) fragile |= ORC_FRAG_THRESHOLD;
            if (v1 > 0.0) {
                s = domain01(v2 / v1, p->ratio_lo, p->ratio_hi);
                if (s > 0.0 && s < 1.0 && v1 < mg->dr) fragile |= ORC_FRAG_RATIO;
            } else {
                s = 0.0;
            }
            if (s >= smax) smax = s;
        }
        count = N;
        table_at(r.lut, r.M, smax, out);
        if (p->mip_alpha == 1) out[3] = 1.0;
    } else if (p->mode <= ORC_MIPRGB) {
        /* Eq. MIP with '>=': a later sample wins a tie (Alg. MIP0, MIP1, MIP_RGB). */
        double smax = -INFINITY;
        int64_t kmax = -1;
        for (int64_t k = 0; k < N; ++k) {
            int exact;
            double s = filter_s(p, ray_value(&r, r.V, k, 0), mg->dv, &fragile, &exact);
            sbuf[k] = s;
            ebuf[k] = (uint8_t)exact;
            if (s >= smax) { smax = s; kmax = k; }
        }
        count = N;
        if (p->mode != ORC_MIP0) {
            /* the colour depends on where the maximum is: a near tie could move it */
            double qm[3];
            ray_point(&r, kmax, qm);
            for (int64_t k = 0; k < N; ++k) {
                if (k == kmax) continue;
                double gap = smax - sbuf[k];
                if (gap >= mg->ds) continue;
                if (gap == 0.0 && ebuf[k] && ebuf[kmax]) continue;
                if (gap == 0.0 && p->box_arm == 0) {
                    double qk[3];
                    ray_point(&r, k, qk);
                    int same = 1;
                    const int32_t n[3] = {r.nx, r.ny, r.nz};
                    for (int a = 0; a < 3; ++a)
                        if (clampd(qk[a], 0.0, n[a] - 1.0) != clampd(qm[a], 0.0, n[a] - 1.0)) same = 0;
                    if (same) continue;
                }
                fragile |= ORC_FRAG_ARGMAX;
                break;
            }
            /* The other reading of a near tie: any sample within ds of the maximum is an
             * arg-max the '>=' of Eq. MIP could have kept under rounding. */
            if (forced >= 0) {
                if (forced >= N || smax - sbuf[forced] >= mg->ds) fragile |= ORC_NOT_CANDIDATE;
                if (forced < N) kmax = forced;
            }
        }
        double alpha;
        if (p->mode == ORC_MIP0) {
            table_at(r.lut, r.M, smax, out);
            alpha = out[3];
        } else {
            double loc[3];
            ray_loc(&r, kmax, loc);
            if (p->mode == ORC_MIP1) {
                table_at(r.lut, r.M, loc[2], out);
            } else {
                out[0] = loc[2];  /* r = velocity */
                out[1] = loc[1];  /* g = Dec */
                out[2] = loc[0];  /* b = RA */
            }
            alpha = smax;
        }
        if (p->mip_alpha == 1) {
            alpha = 1.0;
        } else if (p->mip_alpha == 2) {
            /* Workaround of the Discussion (Section 5.7): transparent only where the
             * maximum is at or below the minimum threshold, opaque elsewhere. */
            double sthr = domain01(p->min_t, p->lo, p->hi);
            if (fabs(smax - sthr) < mg->ds) fragile |= ORC_FRAG_ARGMAX;
            if (smax > sthr) alpha = 1.0;
        }
        out[3] = alpha;
    } else {
        /* Alg. AVIP0 / AVIP1 / AVIP_RGB: front-to-back compositing with the weighting factor
         * k; the ray stops after the sample whose accumulated alpha exceeds 0.99 (ert). */
        double T[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t k = 0; k < N; ++k) {
            int exact;
            double s = filter_s(p, ray_value(&r, r.V, k, 0), mg->dv, &fragile, &exact);
            double tab[4], colour[3], a;
            table_at(r.lut, r.M, s, tab);
            if (p->mode == ORC_AVIP0) {
                colour[0] = tab[0]; colour[1] = tab[1]; colour[2] = tab[2];
            } else {
                double loc[3];
                ray_loc(&r, k, loc);
                if (p->mode == ORC_AVIP1) {
                    double c2[4];
                    table_at(r.lut, r.M, loc[2], c2);
                    colour[0] = c2[0]; colour[1] = c2[1]; colour[2] = c2[2];
                } else {
                    colour[0] = loc[2]; colour[1] = loc[1]; colour[2] = loc[0];
                }
            }
            /* Reading: the opacity weight is k*s (Alg. AVIP0 "val x k"), or k*table(s).a
             * when the transfer function supplies an opacity (Eq. AVIP's k proportional to
             * a function of v). */
            a = p->k * (p->opacity_from_lut ? tab[3] : s);
            double a1 = T[3];
            double a2 = a * (1.0 - a1);
            double al = a1 + a2;
            if (al < p->min_val) al = p->min_val;
            for (int ch = 0; ch < 3; ++ch) T[ch] = T[ch] * (a1 / al) + colour[ch] * (a2 / al);
            T[3] = al;
            ++count;
            if (forced >= 0) {
                if (count >= forced) break;
                continue;
            }
            if (fabs(al - p->ert) < mg->da) fragile |= ORC_FRAG_ERT;
            if (al > p->ert) break;
        }
        out[0] = T[0]; out[1] = T[1]; out[2] = T[2]; out[3] = T[3];
    }
    *frag_out = (uint8_t)fragile;
    if (ns_out) *ns_out = (int32_t)count;
}

static void render_pixel(const ray_ctx* base, const orc_camera* cam, int32_t px, int32_t py,
                         int32_t forced, double out[4], uint8_t* frag_out, int32_t* ns_out,
                         double* sbuf, uint8_t* ebuf) {
    render_core(base, cam, px, py, 0, forced, out, frag_out, ns_out, sbuf, ebuf);
    if (base->mg->pv > 0.0 || base->mg->pp > 0.0) {
        /* conditioning probe: move every sample position and value and watch the output */
        double worst = 0.0;
        for (int pert = 1; pert <= 4; ++pert) {
            if (pert == 3 && !base->V2) continue;
            double alt[4];
            uint8_t f;
            render_core(base, cam, px, py, pert, forced, alt, &f, NULL, sbuf, ebuf);
            for (int ch = 0; ch < 4; ++ch) {
                double dlt = fabs(alt[ch] - out[ch]);
                if (dlt > worst) worst = dlt;
            }
        }
        if (worst > base->mg->pt) *frag_out |= ORC_FRAG_COND;
    }
}

static int check_common(int32_t nx, int32_t ny, int32_t nz, const orc_camera* cam,
                        int32_t M, const orc_params* p) {
    if (nx < 1 || ny < 1 || nz < 1 || !cam || cam->width < 1 || cam->height < 1) return 1;
    if (M < 2 || !p || !(p->dt > 0.0)) return 1;
    if (p->mode < 0 || p->mode > ORC_AVIPRGB) return 1;
    if (p->ratio && (p->box_arm != 0 || p->mode != ORC_MIP0)) return 1;
    if (p->star_n < 0 || p->star_n > 4) return 1;
    if (p->star_n > 0 && (p->box_arm != 0 || p->ratio)) return 1;
    return 0;
}

int orc_render(const double* V, const double* V2, int32_t nx, int32_t ny, int32_t nz,
               const orc_camera* cam, const double* lut, int32_t M, const orc_params* p,
               const orc_margins* mg, int64_t npix, const int64_t* pix,
               const int32_t* forced_n, double* rgba, uint8_t* fragile, int32_t* nsamples,
               int32_t nthreads) {
    if (!V || check_common(nx, ny, nz, cam, M, p) || !mg || !rgba || !fragile) return 1;
    if (p->ratio && !V2) return 1;
    const int64_t npx = (int64_t)cam->width * cam->height;
    if (!pix) npix = npx;
    ray_ctx base;
    memset(&base, 0, sizeof base);
    base.V = V; base.V2 = V2; base.nx = nx; base.ny = ny; base.nz = nz;
    base.lut = lut; base.M = M; base.p = p; base.mg = mg;
    double diag = sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
    int64_t maxN = (int64_t)ceil(diag / p->dt) + 4;
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double* sbuf = (double*)malloc(sizeof(double) * (size_t)maxN);
        uint8_t* ebuf = (uint8_t*)malloc((size_t)maxN);
        if (!sbuf || !ebuf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < npix; ++i) {
                int64_t id = pix ? pix[i] : i;
                if (id < 0 || id >= npx) { fragile[i] = ORC_FRAG_COUNT; continue; }
                int32_t px = (int32_t)(id % cam->width), py = (int32_t)(id / cam->width);
                render_pixel(&base, cam, px, py, forced_n ? forced_n[i] : -1, rgba + 4 * i,
                             fragile + i, nsamples ? nsamples + i : NULL, sbuf, ebuf);
            }
        }
        free(sbuf);
        free(ebuf);
    }
    return bad;
}

/* ---------------------------------------------------------------------------------------
 * Reverse mode of AVIP0 with a piecewise-linear transfer function (every sample stored).
 * Conventions: the termination index, the filter branches and the table interval are held
 * at their forward values; the minVal clamp passes no gradient when it is active;
 * d s / d v = 1/(hi-lo) strictly inside (0, 1), else 0.
 * ------------------------------------------------------------------------------------- */
typedef struct {
    double s, a, a1, al, C0[3], C1[3], col[3];
    int64_t idx[8];
    double w[8];
    double dsdv;
} grad_rec;

static void trilinear_stencil(int32_t nx, int32_t ny, int32_t nz, const double q[3],
                              int64_t idx[8], double w[8]) {
    double x = clampd(q[0], 0.0, nx - 1.0);
    double y = clampd(q[1], 0.0, ny - 1.0);
    double z = clampd(q[2], 0.0, nz - 1.0);
    int64_t i0 = (int64_t)floor(x), j0 = (int64_t)floor(y), l0 = (int64_t)floor(z);
    int64_t i[2] = {i0, i0 + 1 < nx ? i0 + 1 : nx - 1};
    int64_t j[2] = {j0, j0 + 1 < ny ? j0 + 1 : ny - 1};
    int64_t l[2] = {l0, l0 + 1 < nz ? l0 + 1 : nz - 1};
    double fx = x - (double)i0, fy = y - (double)j0, fz = z - (double)l0;
    double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
    int c = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx, ++c) {
                idx[c] = (l[dz] * (int64_t)ny + j[dy]) * (int64_t)nx + i[dx];
                w[c] = wx[dx] * wy[dy] * wz[dz];
            }
}

int orc_render_grad(const double* V, int32_t nx, int32_t ny, int32_t nz,
                    const orc_camera* cam, const double* tf, int32_t M, const orc_params* p,
                    int64_t npix, const int64_t* pix, const double* grad_rgba,
                    double* rgba, double* grad_tf, double* grad_vox) {
    if (!V || check_common(nx, ny, nz, cam, M, p) || !tf || !grad_rgba || !rgba) return 1;
    if (p->mode != ORC_AVIP0 || p->filter != ORC_FILTER_NONE || p->box_arm != 0 || p->ratio ||
        p->star_n != 0)
        return 1;
    const int64_t npx = (int64_t)cam->width * cam->height;
    if (!pix) npix = npx;
    double diag = sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
    int64_t maxN = (int64_t)ceil(diag / p->dt) + 4;
    grad_rec* rec = (grad_rec*)malloc(sizeof(grad_rec) * (size_t)maxN);
    if (!rec) return 2;
    for (int64_t pi = 0; pi < npix; ++pi) {
        int64_t id = pix ? pix[pi] : pi;
        double* out = rgba + 4 * pi;
        out[0] = out[1] = out[2] = out[3] = 0.0;
        if (id < 0 || id >= npx) continue;
        double o[3], d[3], t0, t1;
        orc_pixel_ray(cam, (int32_t)(id % cam->width), (int32_t)(id / cam->width), o, d);
        if (!orc_ray_box(nx, ny, nz, o, d, &t0, &t1)) continue;
        int64_t N = (int64_t)ceil((t1 - t0) / p->dt);
        double T[4] = {0, 0, 0, 0};
        int64_t K = 0;
        for (int64_t k = 0; k < N; ++k) {
            grad_rec* g = &rec[K];
            double q[3], t = t0 + (double)k * p->dt;
            for (int a = 0; a < 3; ++a) q[a] = o[a] + t * d[a];
            double v = orc_trilinear(V, nx, ny, nz, q);
            trilinear_stencil(nx, ny, nz, q, g->idx, g->w);
            double u = p->hi > p->lo ? (v - p->lo) / (p->hi - p->lo) : 0.0;
            double s = clampd(u, 0.0, 1.0);
            g->dsdv = (p->hi > p->lo && u > 0.0 && u < 1.0) ? 1.0 / (p->hi - p->lo) : 0.0;
            double tab[4];
            table_at(tf, M, s, tab);
            g->s = s;
            g->a = p->k * tab[3];
            g->col[0] = tab[0]; g->col[1] = tab[1]; g->col[2] = tab[2];
            g->a1 = T[3];
            double a2 = g->a * (1.0 - g->a1);
            double al = g->a1 + a2;
            if (al < p->min_val) al = p->min_val;
            g->al = al;
            for (int ch = 0; ch < 3; ++ch) {
                g->C0[ch] = T[ch];
                T[ch] = T[ch] * (g->a1 / al) + g->col[ch] * (a2 / al);
                g->C1[ch] = T[ch];
            }
            T[3] = al;
            ++K;
            if (al > p->ert) break;
        }
        out[0] = T[0]; out[1] = T[1]; out[2] = T[2]; out[3] = T[3];
        double gC[3] = {grad_rgba[4 * pi + 0], grad_rgba[4 * pi + 1], grad_rgba[4 * pi + 2]};
        double gA = grad_rgba[4 * pi + 3];
        for (int64_t k = K - 1; k >= 0; --k) {
            const grad_rec* g = &rec[k];
            double a1 = g->a1, a2 = g->a * (1.0 - a1), al = g->al;
            int active = (a1 + a2 >= p->min_val);
            double g_al = gA;
            for (int ch = 0; ch < 3; ++ch) g_al -= gC[ch] * g->C1[ch] / al;
            double g_a2 = active ? g_al : 0.0, g_a1 = active ? g_al : 0.0;
            double gcol[3];
            for (int ch = 0; ch < 3; ++ch) {
                g_a2 += gC[ch] * g->col[ch] / al;
                g_a1 += gC[ch] * g->C0[ch] / al;
                gcol[ch] = gC[ch] * a2 / al;
            }
            g_a1 += g_a2 * (-g->a);
            double g_a = g_a2 * (1.0 - a1);
            /* table(s): interval j0 = min(floor(s (M-1)), M-2), weight f */
            double x = g->s * (M - 1);
            int64_t j0 = (int64_t)floor(x);
            if (j0 > M - 2) j0 = M - 2;
            if (j0 < 0) j0 = 0;
            double f = x - (double)j0;
            double gch[4] = {gcol[0], gcol[1], gcol[2], p->k * g_a};
            double gs = 0.0;
            for (int ch = 0; ch < 4; ++ch) {
                grad_tf[4 * j0 + ch] += (1.0 - f) * gch[ch];
                grad_tf[4 * (j0 + 1) + ch] += f * gch[ch];
                gs += gch[ch] * (tf[4 * (j0 + 1) + ch] - tf[4 * j0 + ch]) * (M - 1);
            }
            double gv = gs * g->dsdv;
            if (grad_vox && gv != 0.0)
                for (int c = 0; c < 8; ++c) grad_vox[g->idx[c]] += gv * g->w[c];
            for (int ch = 0; ch < 3; ++ch) gC[ch] = gC[ch] * a1 / al;
            gA = g_a1;
        }
    }
    free(rec);
    return 0;
}

/* ---------------------------------------------------------------------------------------
 * Section 4.2: the 3D Gaussian is applied as the same 1D kernel successively along each
 * axis (separable), here with clamp-to-edge at the borders and centred odd taps.
 * ------------------------------------------------------------------------------------- */
static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

int orc_smooth(const double* V, int32_t nx, int32_t ny, int32_t nz, const double* g,
               int32_t T, double* out, double* tmp, int32_t nthreads) {
    if (!V || !g || !out || !tmp || T < 1 || (T % 2) == 0 || nx < 1 || ny < 1 || nz < 1)
        return 1;
    const int64_t r = T / 2, sx = 1, sy = nx, sz = (int64_t)nx * ny;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* along x: V -> out */
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int64_t j = 0; j < T; ++j)
                    acc += g[j] * V[z * sz + y * sy + clampi(x + j - r, 0, nx - 1) * sx];
                out[z * sz + y * sy + x] = acc;
            }
    /* along y: out -> tmp */
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int64_t j = 0; j < T; ++j)
                    acc += g[j] * out[z * sz + clampi(y + j - r, 0, ny - 1) * sy + x];
                tmp[z * sz + y * sy + x] = acc;
            }
    /* along z: tmp -> out */
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int64_t j = 0; j < T; ++j)
                    acc += g[j] * tmp[clampi(z + j - r, 0, nz - 1) * sz + y * sy + x];
                out[z * sz + y * sy + x] = acc;
            }
    return 0;
}

int orc_smooth_at(const double* V, int32_t nx, int32_t ny, int32_t nz, const double* g,
                  int32_t T, int64_t npts, const int64_t* idx, double* out) {
    if (!V || !g || !idx || !out || T < 1 || (T % 2) == 0) return 1;
    const int64_t r = T / 2, sz = (int64_t)nx * ny, nvox = sz * nz;
    for (int64_t i = 0; i < npts; ++i) {
        if (idx[i] < 0 || idx[i] >= nvox) return 1;
        int64_t z = idx[i] / sz, y = (idx[i] % sz) / nx, x = idx[i] % nx;
        double acc = 0.0;
        for (int64_t c = 0; c < T; ++c) {
            int64_t zz = clampi(z + c - r, 0, nz - 1);
            for (int64_t b = 0; b < T; ++b) {
                int64_t yy = clampi(y + b - r, 0, ny - 1);
                for (int64_t a = 0; a < T; ++a) {
                    int64_t xx = clampi(x + a - r, 0, nx - 1);
                    acc += g[c] * g[b] * g[a] * V[zz * sz + yy * nx + xx];
                }
            }
        }
        out[i] = acc;
    }
    return 0;
}

/* Section 4.5, method 2 without interpolation: ratio of two co-registered spectral windows,
 * voxel by voxel: window b over window a where a > 0, else DATAMIN; each window first
 * clipped at its own minimum threshold (values below -> DATAMIN). */
int orc_line_ratio(const double* V, int32_t nx, int32_t ny, int32_t nz, int32_t z0a,
                   int32_t z0b, int32_t nzw, double min_t_a, double min_t_b, double datamin,
                   double* out) {
    if (!V || !out || nzw < 1 || z0a < 0 || z0b < 0 || z0a + nzw > nz || z0b + nzw > nz)
        return 1;
    const int64_t plane = (int64_t)nx * ny;
    for (int64_t j = 0; j < nzw; ++j)
        for (int64_t i = 0; i < plane; ++i) {
            double a = V[(z0a + j) * plane + i];
            double b = V[(z0b + j) * plane + i];
            if (a < min_t_a) a = datamin;
            if (b < min_t_b) b = datamin;
            out[j * plane + i] = a > 0.0 ? b / a : datamin;
        }
    return 0;
}

/* Section 2.2: the zeroth moment integrates each spectrum (Eq. mom0, the channel sum times the
 * channel width), the first moment is its intensity-weighted mean channel (Eq. mom1), and the
 * argmax variant returns the channel of the spectrum's maximum.  Readings: channels that are
 * not finite or fall outside [min_t, max_t] do not count (like clipped samples); ties in the
 * maximum go to the later channel, as in the MIP rule of Eq. MIP (v_i >= c_{i-1}). */
int orc_moments(const double* V, int32_t nx, int32_t ny, int32_t nz, int32_t z0, int32_t nzw,
                double dv, double min_t, double max_t, double* m0, double* m1, int32_t* amax) {
    if (!V || !m0 || !m1 || !amax || nzw < 1 || z0 < 0 || z0 + nzw > nz) return 1;
    const int64_t plane = (int64_t)nx * ny;
    for (int64_t i = 0; i < plane; ++i) {
        double s0 = 0.0, s1 = 0.0, best = 0.0;
        int32_t arg = -1;
        for (int32_t z = z0; z < z0 + nzw; ++z) {
            const double v = V[z * plane + i];
            if (!isfinite(v) || v < min_t || v > max_t) continue;
            s0 += v;
            s1 += (double)z * v;
            if (arg < 0 || v >= best) {
                best = v;
                arg = z;
            }
        }
        m0[i] = dv * s0;
        m1[i] = (arg >= 0 && s0 != 0.0) ? s1 / s0 : NAN;
        amax[i] = arg;
    }
    return 0;
}
