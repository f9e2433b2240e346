// C ABI of libsvr: argument validation, ownership of the opaque handles, and dispatch to the
// kernel launchers.  Nothing is enqueued before every argument has been checked.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "common.h"

namespace svr {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

svr_status hip_fail(hipError_t e, const char* what) {
    if (e == hipSuccess) return SVR_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return SVR_EHIP;
}

// launchers (other translation units)
size_t minmax_partial_floats();
svr_status launch_minmax(const svr_cube_view& c, float* partial, float* out, int raw,
                         int out_dtype, float nan_fill, hipStream_t stream);
svr_status launch_minmax_noalloc(const svr_cube_view& c, float* out, hipStream_t stream);
svr_status launch_export(const VolDesc& d, void* out, hipStream_t stream);
svr_status launch_upload(const svr_cube_view& c, const VolDesc& d, float* aux, float nan_fill,
                         hipStream_t stream);
svr_status launch_render(const svr_volume* v, const svr_volume* v2, const svr_camera& cam,
                         const svr_lut& lut, const svr_params& p, float* out,
                         int32_t* samples, hipStream_t stream);
int render_segments(const svr_camera& cam, const VolDesc& v, const svr_params& p);
svr_status launch_smooth(const svr_cube_view& c, const float* taps_host, int ntaps, void* out,
                         void* ws, hipStream_t stream);
bool smooth_fused_taps(int ntaps);
svr_status launch_moments(const svr_cube_view& c, int z0, int nzw, float dv, float lo, float hi,
                          float* m0, float* m1, int32_t* amax, hipStream_t stream);
svr_status launch_line_ratio(const svr_cube_view& c, int z0a, int z0b, int nzw, float min_a,
                             float min_b, float datamin, float* out, hipStream_t stream);

#define SVR_CHECK(cond, ...)            \
    do {                                \
        if (!(cond)) {                  \
            set_error(__VA_ARGS__);     \
            return SVR_EINVAL;          \
        }                               \
    } while (0)

static bool finite3(const float* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

svr_status check_view(const svr_cube_view* c, const char* name) {
    SVR_CHECK(c != nullptr, "%s: null cube view", name);
    SVR_CHECK(c->data != nullptr, "%s: null data pointer", name);
    SVR_CHECK(c->dtype >= SVR_F32 && c->dtype <= SVR_BF16, "%s: dtype %d", name, c->dtype);
    SVR_CHECK(c->nx >= 1 && c->ny >= 1 && c->nz >= 1, "%s: dims %d x %d x %d", name, c->nx,
              c->ny, c->nz);
    SVR_CHECK((c->sx == 0 && c->sy == 0 && c->sz == 0) || (c->sx != 0 && c->sy != 0 && c->sz != 0),
              "%s: strides must be all zero (contiguous) or all nonzero", name);
    return SVR_OK;
}

svr_status check_camera(const svr_camera* c) {
    SVR_CHECK(c != nullptr, "null camera");
    SVR_CHECK(c->type == 0 || c->type == 1, "camera type %d (0 parallel, 1 perspective)", c->type);
    SVR_CHECK(c->width >= 1 && c->height >= 1 && c->width <= 32768 && c->height <= 32768,
              "image %d x %d", c->width, c->height);
    SVR_CHECK(finite3(c->eye) && finite3(c->U) && finite3(c->V) && finite3(c->W),
              "camera vectors must be finite");
    SVR_CHECK(c->W[0] != 0.0f || c->W[1] != 0.0f || c->W[2] != 0.0f, "camera W is zero");
    return SVR_OK;
}

svr_status check_lut(const svr_lut* l) {
    SVR_CHECK(l != nullptr && l->rgba != nullptr, "null colour table");
    SVR_CHECK(aligned_to(l->rgba, 16), "colour table not 16-byte aligned");
    SVR_CHECK(l->n >= 2 && l->n <= SVR_MAX_LUT, "colour table size %d", l->n);
    return SVR_OK;
}

svr_status check_params(const svr_params* p, const svr_volume* v) {
    SVR_CHECK(p != nullptr, "null params");
    SVR_CHECK(p->mode >= SVR_MIP0 && p->mode <= SVR_AVIPRGB, "mode %d", p->mode);
    SVR_CHECK(p->filter >= SVR_FILTER_NONE && p->filter <= SVR_FILTER_SCALE, "filter %d", p->filter);
    SVR_CHECK(p->box_arm >= 0 && p->box_arm <= SVR_MAX_BOX_ARM, "box_arm %d", p->box_arm);
    SVR_CHECK(p->mip_alpha >= 0 && p->mip_alpha <= 2, "mip_alpha %d", p->mip_alpha);
    SVR_CHECK(p->ratio >= 0 && p->ratio <= 2, "ratio %d", p->ratio);
    SVR_CHECK(p->opacity_from_lut == 0 || p->opacity_from_lut == 1, "opacity_from_lut %d",
              p->opacity_from_lut);
    SVR_CHECK(p->k >= 0.0f && p->k <= 1.0f, "k = %g outside [0, 1]", p->k);
    SVR_CHECK(p->min_val > 0.0f && isfinite(p->min_val), "min_val must be > 0");
    SVR_CHECK(isfinite(p->ert), "ert must be finite");
    SVR_CHECK(p->dt > 0.0f && isfinite(p->dt), "dt must be > 0");
    if (v) {
        const double diag = sqrt((double)v->d.nx * v->d.nx + (double)v->d.ny * v->d.ny +
                                 (double)v->d.nz * v->d.nz);
        SVR_CHECK(diag / p->dt < 1.0e8, "dt = %g too small for this volume", p->dt);
    }
    if (p->clim_hi > p->clim_lo)
        SVR_CHECK(isfinite(p->clim_lo) && isfinite(p->clim_hi), "clim must be finite");
    SVR_CHECK(!isnan(p->min_t) && !isnan(p->max_t) && !isnan(p->min_t2) && !isnan(p->max_t2),
              "thresholds must not be NaN");
    if (p->filter == SVR_FILTER_SCALE)
        SVR_CHECK(isfinite(p->min_t) && isfinite(p->max_t) && p->min_t < p->max_t,
                  "domain scaling needs finite min_t < max_t");
    SVR_CHECK(p->star_n >= 0 && p->star_n <= SVR_MAX_STAR, "star_n %d", p->star_n);
    if (p->star_n > 0) {
        SVR_CHECK(p->box_arm == 0 && p->ratio == 0,
                  "the in-ray Gaussian (star_n > 0) takes box_arm 0 and ratio 0");
        SVR_CHECK(isfinite(p->star_c0), "star_c0 must be finite");
        for (int k = 0; k < p->star_n; ++k)
            SVR_CHECK(isfinite(p->star_w[k]) && isfinite(p->star_off[k]) &&
                          p->star_off[k] >= 0.0f && p->star_off[k] <= 64.0f,
                      "star pair %d: offset in [0, 64] and finite weight", k);
    }
    if (p->ratio) {
        SVR_CHECK(p->mode == SVR_MIP0, "line-ratio methods use mode SVR_MIP0");
        SVR_CHECK(p->box_arm == 0, "line-ratio methods take no box smoothing");
        SVR_CHECK(p->filter != SVR_FILTER_SCALE, "line-ratio methods take filter none or clip");
        SVR_CHECK(isfinite(p->ratio_lo) && isfinite(p->ratio_hi), "ratio domain must be finite");
    }
    return SVR_OK;
}

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

static int64_t view_elems_span(const svr_cube_view* c) { return (int64_t)c->nx * c->ny * c->nz; }

}  // namespace svr

using namespace svr;

extern "C" {

const char* svr_status_string(int status) {
    switch (status) {
        case SVR_OK: return "SVR_OK";
        case SVR_EINVAL: return "SVR_EINVAL: invalid argument";
        case SVR_ENOMEM: return "SVR_ENOMEM: out of device memory or workspace too small";
        case SVR_EHIP: return "SVR_EHIP: HIP runtime error";
        case SVR_EUNSUPPORTED: return "SVR_EUNSUPPORTED: not supported";
        default: return "unknown svr_status";
    }
}

const char* svr_last_error(void) { return g_err; }

const char* svr_version(void) { return "svr 1.0 gfx950"; }

svr_status svr_minmax(const svr_cube_view* cube, float* lo_hi_host, void* stream) {
    svr_status st = check_view(cube, "svr_minmax");
    if (st) return st;
    SVR_CHECK(lo_hi_host != nullptr, "svr_minmax: null output");
    float* buf = nullptr;
    const size_t n = minmax_partial_floats() + 4;
    hipError_t e = hipMalloc(&buf, n * sizeof(float));
    if (e != hipSuccess) {
        set_error("svr_minmax: hipMalloc: %s", hipGetErrorString(e));
        return SVR_ENOMEM;
    }
    st = launch_minmax(*cube, buf + 4, buf, 1, SVR_F32, NAN, S(stream));
    if (!st) st = hip_fail(hipMemcpyAsync(lo_hi_host, buf, 2 * sizeof(float),
                                          hipMemcpyDeviceToHost, S(stream)), "svr_minmax copy");
    if (!st) st = hip_fail(hipStreamSynchronize(S(stream)), "svr_minmax sync");
    (void)hipFree(buf);
    return st;
}

svr_status svr_minmax_noalloc(const svr_cube_view* cube, float* lo_hi_dev, void* stream) {
    svr_status st = check_view(cube, "svr_minmax_noalloc");
    if (st) return st;
    SVR_CHECK(lo_hi_dev != nullptr, "svr_minmax_noalloc: null output");
    return launch_minmax_noalloc(*cube, lo_hi_dev, S(stream));
}

svr_status svr_volume_create(const svr_cube_view* src, int32_t storage, int32_t brick,
                             float nan_fill, void* stream, svr_volume** out) {
    svr_status st = check_view(src, "svr_volume_create");
    if (st) return st;
    SVR_CHECK(out != nullptr, "svr_volume_create: null output handle");
    SVR_CHECK(storage >= SVR_F32 && storage <= SVR_BF16, "storage dtype %d", storage);
    if (brick == 0) brick = 8;
    SVR_CHECK(brick == 8 || brick == 16, "brick %d (8 or 16)", brick);
    SVR_CHECK(!isinf(nan_fill), "nan_fill must be finite or NaN");
    if (src->nx > 0xffffff || src->ny > 0xffffff || src->nz > 0xffffff) {
        set_error("svr_volume_create: dims %d x %d x %d: each must be below 2^24", src->nx,
                  src->ny, src->nz);
        return SVR_EUNSUPPORTED;
    }
    VolDesc d = make_voldesc(src->nx, src->ny, src->nz, storage, brick);
    const uint64_t nbricks = (uint64_t)d.nbx * d.nby * d.nbz;
    const uint64_t elems = nbricks * d.pitch;
    if (elems >= (1ull << 32) || nbricks >= (1ull << 24)) {
        set_error("volume of %llu stored elements exceeds 2^32", (unsigned long long)elems);
        return SVR_EUNSUPPORTED;
    }
    const size_t esize = storage == SVR_F32 ? 4 : 2;
    svr_volume* v = new (std::nothrow) svr_volume;
    if (!v) return SVR_ENOMEM;
    v->mem = nullptr;
    v->aux = nullptr;
    v->bytes = (int64_t)(elems * esize);
    (void)hipGetDevice(&v->device);
    hipError_t e = hipMalloc(&v->mem, elems * esize);
    if (e == hipSuccess)
        e = hipMalloc((void**)&v->aux, (minmax_partial_floats() + 4) * sizeof(float));
    if (e != hipSuccess) {
        if (v->mem) (void)hipFree(v->mem);
        delete v;
        set_error("svr_volume_create: hipMalloc: %s", hipGetErrorString(e));
        return SVR_ENOMEM;
    }
    v->bytes += (int64_t)((minmax_partial_floats() + 4) * sizeof(float));
    d.data = v->mem;
    d.clim = v->aux;
    v->d = d;
    st = launch_upload(*src, v->d, v->aux, nan_fill, S(stream));
    if (st) {
        (void)hipFree(v->mem);
        (void)hipFree(v->aux);
        delete v;
        return st;
    }
    *out = v;
    return SVR_OK;
}

svr_status svr_volume_upload(svr_volume* vol, const svr_cube_view* src, float nan_fill,
                             void* stream) {
    SVR_CHECK(vol != nullptr, "svr_volume_upload: null volume");
    svr_status st = check_view(src, "svr_volume_upload");
    if (st) return st;
    SVR_CHECK(src->nx == vol->d.nx && src->ny == vol->d.ny && src->nz == vol->d.nz,
              "svr_volume_upload: dims %d x %d x %d differ from the volume's", src->nx, src->ny,
              src->nz);
    SVR_CHECK(!isinf(nan_fill), "nan_fill must be finite or NaN");
    return launch_upload(*src, vol->d, vol->aux, nan_fill, S(stream));
}

svr_status svr_volume_destroy(svr_volume* vol) {
    if (!vol) return SVR_OK;
    hipError_t e1 = hipFree(vol->mem);
    hipError_t e2 = hipFree(vol->aux);
    delete vol;
    if (e1 != hipSuccess) return hip_fail(e1, "svr_volume_destroy");
    return hip_fail(e2, "svr_volume_destroy");
}

svr_status svr_volume_info(const svr_volume* vol, int32_t* dims_zyx, int32_t* storage,
                           int32_t* brick, int64_t* bytes) {
    SVR_CHECK(vol != nullptr, "null volume");
    if (dims_zyx) {
        dims_zyx[0] = vol->d.nz;
        dims_zyx[1] = vol->d.ny;
        dims_zyx[2] = vol->d.nx;
    }
    if (storage) *storage = vol->d.dtype;
    if (brick) *brick = vol->d.brick;
    if (bytes) *bytes = vol->bytes;
    return SVR_OK;
}

svr_status svr_volume_clim(const svr_volume* vol, float* lo_hi_host, void* stream) {
    SVR_CHECK(vol != nullptr && lo_hi_host != nullptr, "null argument");
    svr_status st = hip_fail(hipMemcpyAsync(lo_hi_host, vol->aux, 2 * sizeof(float),
                                            hipMemcpyDeviceToHost, S(stream)), "clim copy");
    if (st) return st;
    return hip_fail(hipStreamSynchronize(S(stream)), "clim sync");
}

svr_status svr_volume_export(const svr_volume* vol, void* out, void* stream) {
    SVR_CHECK(vol != nullptr && out != nullptr, "null argument");
    return launch_export(vol->d, out, S(stream));
}

svr_status svr_params_validate(const svr_params* params) { return check_params(params, nullptr); }

svr_status svr_render(const svr_volume* vol, const svr_volume* vol2, const svr_camera* cam,
                      const svr_lut* lut, const svr_params* params, float* rgba_out,
                      int32_t* samples_out, void* stream) {
    SVR_CHECK(vol != nullptr, "svr_render: null volume");
    svr_status st;
    if ((st = check_camera(cam))) return st;
    if ((st = check_lut(lut))) return st;
    if ((st = check_params(params, vol))) return st;
    SVR_CHECK(rgba_out != nullptr, "svr_render: null output");
    SVR_CHECK(aligned_to(rgba_out, 16), "svr_render: output not 16-byte aligned");
    SVR_CHECK(aligned_to(samples_out, 4), "svr_render: sample counts not 4-byte aligned");
    if (params->ratio) {
        SVR_CHECK(vol2 != nullptr, "svr_render: line-ratio methods need vol2");
        SVR_CHECK(vol2->d.nx == vol->d.nx && vol2->d.ny == vol->d.ny && vol2->d.nz == vol->d.nz,
                  "svr_render: vol2 dims differ from vol");
        SVR_CHECK(vol2->d.dtype == vol->d.dtype && vol2->d.brick == vol->d.brick,
                  "svr_render: vol2 storage/brick differ from vol");
    }
    return launch_render(vol, params->ratio ? vol2 : nullptr, *cam, *lut, *params, rgba_out,
                         samples_out, S(stream));
}

svr_status svr_render_segments(const svr_volume* vol, const svr_camera* cam,
                               const svr_params* params, int32_t* segments) {
    SVR_CHECK(vol != nullptr && segments != nullptr, "svr_render_segments: null argument");
    svr_status st;
    if ((st = check_camera(cam))) return st;
    if ((st = check_params(params, vol))) return st;
    *segments = render_segments(*cam, vol->d, *params);
    return SVR_OK;
}

svr_status svr_smooth_workspace(const svr_cube_view* in, int32_t ntaps, size_t* bytes) {
    svr_status st = check_view(in, "svr_smooth_workspace");
    if (st) return st;
    SVR_CHECK(bytes != nullptr, "null output");
    SVR_CHECK(ntaps >= 1 && ntaps <= SVR_MAX_TAPS && (ntaps % 2) == 1,
              "svr_smooth_workspace: ntaps = %d (odd, <= %d)", ntaps, SVR_MAX_TAPS);
    *bytes = smooth_fused_taps(ntaps) ? 0 : 2 * (size_t)view_elems_span(in) * sizeof(float);
    return SVR_OK;
}

svr_status svr_smooth(const svr_cube_view* in, const float* taps_host, int32_t ntaps,
                      void* out, void* workspace, size_t workspace_bytes, void* stream) {
    svr_status st = check_view(in, "svr_smooth");
    if (st) return st;
    if (!(in->sx == 0 && in->sy == 0 && in->sz == 0)) {
        set_error("svr_smooth: input must be C-contiguous");
        return SVR_EUNSUPPORTED;
    }
    SVR_CHECK(taps_host != nullptr, "svr_smooth: null taps");
    SVR_CHECK(ntaps >= 1 && ntaps <= SVR_MAX_TAPS && (ntaps % 2) == 1,
              "svr_smooth: ntaps = %d (odd, <= %d)", ntaps, SVR_MAX_TAPS);
    for (int j = 0; j < ntaps; ++j)
        SVR_CHECK(isfinite(taps_host[j]), "svr_smooth: tap %d not finite", j);
    SVR_CHECK(out != nullptr, "svr_smooth: null output");
    SVR_CHECK(out != in->data, "svr_smooth: out must not alias the input");
    SVR_CHECK((int64_t)in->ny * in->nz < (1ll << 31) && in->nz <= 65535 &&
                  (int64_t)in->nx * in->ny < (1ll << 31),
              "svr_smooth: cube too large for the launch grid");
    const size_t need =
        smooth_fused_taps(ntaps) ? 0 : 2 * (size_t)view_elems_span(in) * sizeof(float);
    SVR_CHECK(need == 0 || workspace != nullptr, "svr_smooth: null workspace");
    if (workspace_bytes < need) {
        set_error("svr_smooth: workspace %zu < %zu bytes", workspace_bytes, need);
        return SVR_ENOMEM;
    }
    return launch_smooth(*in, taps_host, ntaps, out, workspace, S(stream));
}

svr_status svr_line_ratio(const svr_cube_view* cube, int32_t z0_a, int32_t z0_b, int32_t nz_w,
                          float min_t_a, float min_t_b, float datamin, float* ratio_out,
                          void* stream) {
    svr_status st = check_view(cube, "svr_line_ratio");
    if (st) return st;
    SVR_CHECK(nz_w >= 1 && nz_w <= 65535, "svr_line_ratio: window length %d", nz_w);
    SVR_CHECK(z0_a >= 0 && z0_b >= 0 && (int64_t)z0_a + nz_w <= cube->nz &&
                  (int64_t)z0_b + nz_w <= cube->nz,
              "svr_line_ratio: windows [%d, %lld) and [%d, %lld) outside 0..%d", z0_a,
              (long long)z0_a + nz_w, z0_b, (long long)z0_b + nz_w, cube->nz);
    SVR_CHECK(cube->ny <= 65535, "svr_line_ratio: ny too large for the launch grid");
    SVR_CHECK(!isnan(min_t_a) && !isnan(min_t_b) && !isnan(datamin), "svr_line_ratio: NaN argument");
    SVR_CHECK(ratio_out != nullptr, "svr_line_ratio: null output");
    return launch_line_ratio(*cube, z0_a, z0_b, nz_w, min_t_a, min_t_b, datamin, ratio_out,
                             S(stream));
}

svr_status svr_moments(const svr_cube_view* cube, int32_t z0, int32_t nz_w, float dv,
                       float min_t, float max_t, float* m0_out, float* m1_out,
                       int32_t* argmax_out, void* stream) {
    svr_status st = check_view(cube, "svr_moments");
    if (st) return st;
    SVR_CHECK(nz_w >= 1 && z0 >= 0 && (int64_t)z0 + nz_w <= cube->nz,
              "svr_moments: window [%d, %lld) outside 0..%d", z0, (long long)z0 + nz_w,
              cube->nz);
    SVR_CHECK(cube->ny <= 65535, "svr_moments: ny too large for the launch grid");
    SVR_CHECK(!isnan(dv) && !isnan(min_t) && !isnan(max_t), "svr_moments: NaN argument");
    SVR_CHECK(min_t <= max_t, "svr_moments: min_t %g > max_t %g", (double)min_t, (double)max_t);
    SVR_CHECK(m0_out != nullptr || m1_out != nullptr || argmax_out != nullptr,
              "svr_moments: no output");
    return launch_moments(*cube, z0, nz_w, dv, min_t, max_t, m0_out, m1_out, argmax_out,
                          S(stream));
}

svr_status svr_sync(void* stream) {
    svr_status st = hip_fail(hipStreamSynchronize(S(stream)), "svr_sync");
    if (st) return st;
    return hip_fail(hipGetLastError(), "svr_sync (pending error)");
}

}  // extern "C"
