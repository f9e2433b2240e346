// Per-ray march shared by the single-image and the batched kernels (identical arithmetic).
#pragma once

#include "sampler.h"

namespace svr {

struct RenderArgs {
    VolDesc v, v2;
    svr_camera cam;
    const float4* lut;
    int32_t lut_n;
    svr_params p;
    float4* out;
    int32_t* samples;
    int32_t tiles_x, nblocks;
};

// filter() of Alg. 1 then the map onto [0, 1] (DATAMIN = lo maps to 0).
struct Filt {
    int kind;
    float lo, inv, mn, mx, sinv;
    __device__ __forceinline__ float operator()(float v) const {
        if (kind == SVR_FILTER_SCALE) return (v > mx || v < mn) ? 0.0f : (v - mn) * sinv;
        if (kind == SVR_FILTER_CLIP && (v < mn || v > mx)) v = lo;
        return __saturatef((v - lo) * inv);
    }
};

// Sample source along one ray: position k -> raw value, with optional box mean along the
// ray.  The ring keeps the last 2a+1 raw samples of this lane in LDS (stride = block size).
template <class S>
struct Stream {
    S smp;
    float p0x, p0y, p0z, sx, sy, sz;
    __device__ __forceinline__ float at(float kf) const {
        return smp(fmaf(kf, sx, p0x), fmaf(kf, sy, p0y), fmaf(kf, sz, p0z));
    }
};

template <int MODE, int RATIO, int DT, int C, bool BOX>
__device__ __forceinline__ void march(const RenderArgs& a, const float4* s_lut, float* ring,
                                      const RaySeg& r, const Filt& F, float4& res,
                                      int& count) {
    using Smp = Sampler<DT, C>;
    const Stream<Smp> st{Smp(a.v), r.p0[0], r.p0[1], r.p0[2], r.step[0], r.step[1], r.step[2]};
    const int N = r.n;
    const int n_lut = a.lut_n;
    const int arm = BOX ? a.p.box_arm : 0;
    const int L = 2 * arm + 1;
    const float box_coeff = 1.0f / (float)L;
    int head = 0;
    if (BOX) {
        // samples -arm .. arm-1 fill slots 0 .. L-2
        for (int j = -arm; j < arm; ++j) ring[(j + arm) * kBlock] = st.at((float)j);
    }
    auto value = [&](int k, float kf) -> float {
        if (!BOX) return st.at(kf);
        const int wslot = head == 0 ? L - 1 : head - 1;
        ring[wslot * kBlock] = st.at(kf + (float)arm);
        float sum = 0.0f;
        int idx = head;
        for (int i = 0; i < L; ++i) {
            sum += ring[idx * kBlock];
            idx = idx + 1 == L ? 0 : idx + 1;
        }
        head = head + 1 == L ? 0 : head + 1;
        (void)k;
        return sum * box_coeff;
    };

    if (RATIO == 1) {
        // Line ratio, method 1: per-cube MIP with strict '>' then colourMap(max2/max1).
        const Stream<Smp> st2{Smp(a.v2), r.p0[0], r.p0[1], r.p0[2], r.step[0], r.step[1],
                              r.step[2]};
        const bool clip = a.p.filter == SVR_FILTER_CLIP;
        float m1 = -INFINITY, m2 = -INFINITY, kf = 0.0f;
        for (int k = 0; k < N; ++k, kf += 1.0f) {
            float v1 = st.at(kf), v2 = st2.at(kf);
            if (clip) {
                if (v1 < a.p.min_t || v1 > a.p.max_t) v1 = F.lo;
                if (v2 < a.p.min_t2 || v2 > a.p.max_t2) v2 = F.lo;
            }
            m1 = v1 > m1 ? v1 : m1;
            m2 = v2 > m2 ? v2 : m2;
        }
        count = N;
        if (m1 > 0.0f) {
            const float rr = m2 / m1;
            const float rinv = a.p.ratio_hi > a.p.ratio_lo ? 1.0f / (a.p.ratio_hi - a.p.ratio_lo) : 0.0f;
            res = table(s_lut, n_lut, __saturatef((rr - a.p.ratio_lo) * rinv));
            if (a.p.mip_alpha == 1) res.w = 1.0f;
        }
        return;
    }
    if (RATIO == 2) {
        // Line ratio, method 2: per-sample ratio (DATAMIN -> 0 where cube 1 <= 0), then MIP0.
        const Stream<Smp> st2{Smp(a.v2), r.p0[0], r.p0[1], r.p0[2], r.step[0], r.step[1],
                              r.step[2]};
        const bool clip = a.p.filter == SVR_FILTER_CLIP;
        const float rinv = a.p.ratio_hi > a.p.ratio_lo ? 1.0f / (a.p.ratio_hi - a.p.ratio_lo) : 0.0f;
        float smax = -INFINITY, kf = 0.0f;
        for (int k = 0; k < N; ++k, kf += 1.0f) {
            float v1 = st.at(kf), v2 = st2.at(kf);
            if (clip) {
                if (v1 < a.p.min_t || v1 > a.p.max_t) v1 = F.lo;
                if (v2 < a.p.min_t2 || v2 > a.p.max_t2) v2 = F.lo;
            }
            const float s = v1 > 0.0f ? __saturatef((v2 / v1 - a.p.ratio_lo) * rinv) : 0.0f;
            smax = s >= smax ? s : smax;
        }
        count = N;
        res = table(s_lut, n_lut, smax);
        if (a.p.mip_alpha == 1) res.w = 1.0f;
        return;
    }

    if (MODE <= SVR_MIPRGB) {
        // Eq. MIP, '>=' so a later sample wins a tie; MIP1/MIP_RGB keep the arg-max index.
        float smax = -INFINITY, kf = 0.0f;
        int kmax = 0;
        for (int k = 0; k < N; ++k, kf += 1.0f) {
            const float s = F(value(k, kf));
            if (MODE == SVR_MIP0) {
                smax = s >= smax ? s : smax;
            } else if (s >= smax) {
                smax = s;
                kmax = k;
            }
        }
        count = N;
        float alpha;
        if (MODE == SVR_MIP0) {
            res = table(s_lut, n_lut, smax);
            alpha = res.w;
        } else {
            const float km = (float)kmax;
            const float lx = __saturatef((fmaf(km, r.step[0], r.p0[0]) + 0.5f) / (float)a.v.nx);
            const float ly = __saturatef((fmaf(km, r.step[1], r.p0[1]) + 0.5f) / (float)a.v.ny);
            const float lz = __saturatef((fmaf(km, r.step[2], r.p0[2]) + 0.5f) / (float)a.v.nz);
            if (MODE == SVR_MIP1) {
                res = table(s_lut, n_lut, lz);
            } else {
                res = make_float4(lz, ly, lx, 0.0f);
            }
            alpha = smax;
        }
        if (a.p.mip_alpha == 1) {
            alpha = 1.0f;
        } else if (a.p.mip_alpha == 2) {
            const float sthr = __saturatef((a.p.min_t - F.lo) * F.inv);
            if (smax > sthr) alpha = 1.0f;
        }
        res.w = alpha;
        return;
    }

    // Alg. AVIP0 / AVIP1 / AVIP_RGB: front-to-back compositing, stop after alpha > ert.
    const float kw = a.p.k, minv = a.p.min_val, ert = a.p.ert;
    const bool ofl = a.p.opacity_from_lut != 0;
    const float inx = 1.0f / (float)a.v.nx, iny = 1.0f / (float)a.v.ny, inz = 1.0f / (float)a.v.nz;
    float tr = 0.0f, tg = 0.0f, tb = 0.0f, ta = 0.0f, kf = 0.0f;
    int cnt = 0;
    for (int k = 0; k < N; ++k, kf += 1.0f) {
        const float s = F(value(k, kf));
        float cr, cg, cb, op;
        if (MODE == SVR_AVIP0) {
            const float4 c = table(s_lut, n_lut, s);
            cr = c.x; cg = c.y; cb = c.z;
            op = ofl ? c.w : s;
        } else {
            const float lz = __saturatef((fmaf(kf, r.step[2], r.p0[2]) + 0.5f) * inz);
            if (MODE == SVR_AVIP1) {
                const float4 c = table(s_lut, n_lut, lz);
                cr = c.x; cg = c.y; cb = c.z;
            } else {
                cr = lz;
                cg = __saturatef((fmaf(kf, r.step[1], r.p0[1]) + 0.5f) * iny);
                cb = __saturatef((fmaf(kf, r.step[0], r.p0[0]) + 0.5f) * inx);
            }
            op = ofl ? table(s_lut, n_lut, s).w : s;
        }
        const float a1 = ta;
        const float a2 = kw * op * (1.0f - a1);
        const float al = fmaxf(a1 + a2, minv);
        const float ri = rcp(al);
        const float w1 = a1 * ri, w2 = a2 * ri;
        tr = fmaf(tr, w1, cr * w2);
        tg = fmaf(tg, w1, cg * w2);
        tb = fmaf(tb, w1, cb * w2);
        ta = al;
        ++cnt;
        if (al > ert) break;
    }
    count = cnt;
    res = make_float4(tr, tg, tb, ta);
}

// One ray of Alg. 1 for pixel (px, py): colour-map domain, filter, ray setup, march.
template <int MODE, int RATIO, int DT, int C>
__device__ __forceinline__ void render_ray(const RenderArgs& a, const float4* s_lut, float* ring,
                                           int px, int py, float4& res, int& count) {
    Filt F;
    F.kind = a.p.filter;
    F.lo = a.p.clim_lo;
    float hi = a.p.clim_hi;
    if (!(hi > F.lo)) {
        F.lo = a.v.clim[0];
        hi = a.v.clim[1];
    }
    F.inv = hi > F.lo ? 1.0f / (hi - F.lo) : 0.0f;
    F.mn = a.p.min_t;
    F.mx = a.p.max_t;
    F.sinv = a.p.max_t > a.p.min_t ? 1.0f / (a.p.max_t - a.p.min_t) : 0.0f;
    const RaySeg r = ray_segment(a.cam, px, py, a.v.nx, a.v.ny, a.v.nz, a.p.dt);
    res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    count = 0;
    if (r.n > 0) {
        if (RATIO == 0 && a.p.box_arm > 0)
            march<MODE, RATIO, DT, C, true>(a, s_lut, ring, r, F, res, count);
        else
            march<MODE, RATIO, DT, C, false>(a, s_lut, ring, r, F, res, count);
    }
}

size_t render_lds_bytes(int lut_n, int box_arm, int ratio);

}  // namespace svr
