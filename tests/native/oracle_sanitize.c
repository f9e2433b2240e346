/* Drives every entry point of the FP64 oracle on small ragged inputs, for an
 * AddressSanitizer + UndefinedBehaviorSanitizer build (tests/test_sanitizers.py): any
 * out-of-bounds access, leak or undefined operation aborts with a report.  Values come
 * from a fixed linear congruential sequence; nothing here checks results. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static unsigned long long g_state = 88172645463325252ull;
static double urand(void) {
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) / 9007199254740992.0;
}

static orc_camera camera(int type, int nx, int ny, int nz, int w, int h, double az) {
    orc_camera c;
    memset(&c, 0, sizeof c);
    c.type = type;
    c.width = w;
    c.height = h;
    const double cx = (nx - 1) / 2.0, cy = (ny - 1) / 2.0, cz = (nz - 1) / 2.0;
    const double dx = sin(az), dz = cos(az), r = 2.0 * (nx + ny + nz);
    c.W[0] = dx; c.W[1] = 0.1; c.W[2] = dz;
    c.eye[0] = cx - r * dx; c.eye[1] = cy - 0.1 * r; c.eye[2] = cz - r * dz;
    c.U[0] = dz * (type ? 0.4 : nx); c.U[2] = -dx * (type ? 0.4 : nx);
    c.V[1] = type ? 0.4 : ny;
    return c;
}

int main(void) {
    const int nx = 13, ny = 9, nz = 11, M = 17;
    const size_t nv = (size_t)nx * ny * nz;
    double* V = malloc(nv * sizeof(double));
    double* V2 = malloc(nv * sizeof(double));
    for (size_t i = 0; i < nv; ++i) {
        V[i] = 4.0 * urand() - 1.0;
        V2[i] = 3.0 * urand() - 0.5;
    }
    double lut[4 * M];
    for (int i = 0; i < 4 * M; ++i) lut[i] = urand();
    orc_margins mg = {1e-5, 1e-5, 2e-6, 1e-9, 1e-3, 1e-6, 1e-5, 1e-7};
    const int W = 7, H = 5, npix = W * H;
    double rgba[4 * 35], grad[4 * 35], gtf[4 * M];
    uint8_t frag[35];
    int32_t ns[35], forced[35];
    int64_t pix[35];
    for (int i = 0; i < npix; ++i) {
        pix[i] = (i * 11) % npix;
        forced[i] = i % 9;
        grad[4 * i] = grad[4 * i + 1] = grad[4 * i + 2] = grad[4 * i + 3] = urand() - 0.5;
    }
    double* gvox = calloc(nv, sizeof(double));
    int calls = 0;
    for (int type = 0; type < 2; ++type) {
        for (int mode = 0; mode < 6; ++mode) {
            for (int filt = 0; filt < 3; ++filt) {
                for (int variant = 0; variant < 4; ++variant) {
                    orc_camera c = camera(type, nx, ny, nz, W, H, 0.3 + mode + variant);
                    orc_params p;
                    memset(&p, 0, sizeof p);
                    p.mode = mode;
                    p.filter = filt;
                    p.k = 0.4;
                    p.min_val = 1e-6;
                    p.ert = 0.99;
                    p.lo = -1.0;
                    p.hi = 3.0;
                    p.dt = 0.37;
                    p.min_t = 0.2;
                    p.max_t = 2.5;
                    p.min_t2 = -0.2;
                    p.max_t2 = 2.0;
                    p.ratio_lo = 0.0;
                    p.ratio_hi = 2.0;
                    p.mip_alpha = variant % 3;
                    p.box_arm = variant == 1 ? 2 : 0;
                    if (variant == 2) {
                        p.star_n = 2;
                        p.star_c0 = 0.227;
                        p.star_off[0] = 1.38; p.star_w[0] = 0.316;
                        p.star_off[1] = 3.23; p.star_w[1] = 0.07;
                    }
                    if (variant == 3 && mode == 0 && filt != 2) p.ratio = 1 + (type & 1);
                    p.opacity_from_lut = variant == 3;
                    const int32_t* f = (variant == 0 && mode >= 1) ? forced : NULL;
                    if (orc_render(V, p.ratio ? V2 : NULL, nx, ny, nz, &c, lut, M, &p, &mg,
                                   npix, variant & 1 ? pix : NULL, f, rgba, frag, ns, 1) != 0)
                        return 2;
                    ++calls;
                    if (mode == 3 && filt == 0 && variant == 3) {
                        memset(gtf, 0, sizeof gtf);
                        if (orc_render_grad(V, nx, ny, nz, &c, lut, M, &p, npix, pix, grad, rgba,
                                            gtf, gvox) != 0)
                            return 3;
                        ++calls;
                    }
                }
            }
        }
    }
    /* smoothing, direct triple sum, line ratio, moments */
    const double g7[7] = {0.05, 0.1, 0.2, 0.3, 0.2, 0.1, 0.05};
    double* out = malloc(nv * sizeof(double));
    double* tmp = malloc(nv * sizeof(double));
    if (orc_smooth(V, nx, ny, nz, g7, 7, out, tmp, 1) != 0) return 4;
    int64_t idx[6] = {0, 1, (int64_t)nv - 1, 57, 400, 1000};
    double at[6];
    if (orc_smooth_at(V, nx, ny, nz, g7, 7, 6, idx, at) != 0) return 5;
    double* ratio = malloc((size_t)nx * ny * 4 * sizeof(double));
    if (orc_line_ratio(V, nx, ny, nz, 1, 7, 4, 0.1, -INFINITY, -1.0, ratio) != 0) return 6;
    double m0[13 * 9], m1[13 * 9];
    int32_t amax[13 * 9];
    V[5] = NAN;
    if (orc_moments(V, nx, ny, nz, 2, 8, 1.5, -0.5, 2.5, m0, m1, amax) != 0) return 7;
    /* single-voxel cube and one-pixel image */
    double one = 0.5;
    orc_camera c1 = camera(1, 1, 1, 1, 1, 1, 0.7);
    orc_params p1;
    memset(&p1, 0, sizeof p1);
    p1.mode = 3; p1.k = 0.5; p1.min_val = 1e-6; p1.ert = 0.99; p1.lo = 0.0; p1.hi = 1.0;
    p1.dt = 0.5; p1.ratio_hi = 1.0;
    if (orc_render(&one, NULL, 1, 1, 1, &c1, lut, M, &p1, &mg, 1, NULL, NULL, rgba, frag, ns,
                   1) != 0)
        return 8;
    free(V); free(V2); free(gvox); free(out); free(tmp); free(ratio);
    printf("oracle sanitize driver: %d render calls ok\n", calls + 1);
    return 0;
}
