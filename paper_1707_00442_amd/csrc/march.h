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

__device__ __forceinline__ float sat(float x) { return med3(x, 0.0f, 1.0f); }

// filter() of Alg. 1 then the map onto [0, 1], branch-free.  A value outside [mn, mx]
// maps to s = 0: clipping replaces it by DATAMIN = lo, domain scaling discards it.  Inside,
// s = (v - base) * scale with (base, scale) = (lo, 1/(hi - lo)) for no filter and clipping,
// (minT, 1/(maxT - minT)) for domain scaling.  No filter uses mn = -inf, mx = +inf.
struct Filt {
    float mn, mx, base, scale;
    float lo, inv;  // the colour-map domain (DATAMIN = lo)
    __device__ __forceinline__ float operator()(float v) const {
        const bool out = (v < mn) | (v > mx);
        return out ? 0.0f : sat((v - base) * scale);
    }
};

// Box mean of Section 4.1 along the ray: the mean of the 2a+1 raw samples centred on k,
// from a per-lane ring of the last 2a+1 raw samples in LDS (slot stride = workgroup size).
// The raw stream starts at sample -a; its first 2a values only fill the ring.  Every lane
// pushes every value (the march loop is uniform), so the slot index is uniform.
struct BoxRing {
    float* ring;
    int L, head;
    float coeff;
    __device__ __forceinline__ BoxRing(float* r, int arm)
        : ring(r), L(2 * arm + 1), head(0), coeff(1.0f / (float)(2 * arm + 1)) {}
    // raw value j of the stream; returns true (and the mean) once a full window is in
    __device__ __forceinline__ bool push(int j, float raw, float& mean) {
        if (j < L - 1) {
            ring[j * kBlock] = raw;  // samples -a .. a-1 fill slots 0 .. L-2
            return false;
        }
        const int wslot = head == 0 ? L - 1 : head - 1;
        ring[wslot * kBlock] = raw;  // sample k + a
        float sum = 0.0f;
        int idx = head;
        for (int i = 0; i < L; ++i) {  // oldest (k - a) to newest (k + a)
            sum += ring[idx * kBlock];
            idx = idx + 1 == L ? 0 : idx + 1;
        }
        head = head + 1 == L ? 0 : head + 1;
        mean = sum * coeff;
        return true;
    }
};

// Smoothing of a sample before filter() (Alg. 1): none, the box mean along the ray
// (Section 4.1) or the in-ray 3-axis Gaussian (Section 4.2).  kSmoothAuto compiles both none
// and box into one kernel and picks per launch from box_arm.
enum { kSmoothNone = 0, kSmoothBox = 1, kSmoothStar = 2, kSmoothAuto = 3 };

// Run alive = per_sample(j, value, active) over the n samples k0 + j (j = 0 .. n-1) of a ray,
// the value being the raw sample or its box mean (the raw stream then starts at k0 - arm and
// fills the ring first, so a run of samples gets the means of the whole ray).
template <int SMOOTH, int NS, class S, class Fn>
__device__ __forceinline__ void for_each_value_from(const S& smp, const RaySeg& r, int k0, int n,
                                                    int arm, float* ring, Fn&& per_sample) {
    static_assert(SMOOTH == kSmoothNone || SMOOTH == kSmoothBox, "raw or box values");
    if (SMOOTH == kSmoothNone) {
        drive<NS>(RaySource<S>(smp, r, (float)k0), n, per_sample);
        return;
    }
    BoxRing box(ring, arm);
    const int lead = 2 * arm;
    drive<NS>(RaySource<S>(smp, r, (float)(k0 - arm)), n > 0 ? n + lead : 0,
          [&](int j, float raw, bool active) -> bool {
              float mean;
              if (!box.push(j, raw, mean)) return active;  // still filling the window
              return per_sample(j - lead, mean, active);
          });
}

// Run alive = per_sample(k, value, active) over the ray's samples k = 0 .. N-1, the value
// being the raw sample, its box mean or its in-ray Gaussian.
template <int SMOOTH, int NS, class S, class Fn>
__device__ __forceinline__ void for_each_value(const S& smp, const RaySeg& r, int arm, float* ring,
                                               const svr_params& st, Fn&& per_sample) {
    if constexpr (SMOOTH == kSmoothStar) {  // values complete at fetch time: one ahead is enough
        drive<2>(StarSource<S>(smp, st, r), r.n, per_sample);
    } else {
        for_each_value_from<SMOOTH, NS>(smp, r, 0, r.n, arm, ring, per_sample);
    }
}

// The sample stream of one ray through the bricked volume: feed.run(body) delivers
// alive = body(k, value, active) for k = 0 .. N-1 (raw or smoothed samples).
template <int SMOOTH, int NS, class Smp>
struct GatherFeed {
    const Smp& smp;
    const RaySeg& r;
    int arm;
    float* ring;
    const svr_params& st;
    template <class Fn>
    __device__ __forceinline__ void run(Fn&& body) const {
        for_each_value<SMOOTH, NS>(smp, r, arm, ring, st, body);
    }
};

template <int MODE, class Feed>
__device__ __forceinline__ void march_tf(const RenderArgs& a, const float4* s_lut,
                                         const RaySeg& r, const Filt& F, Feed& feed,
                                         float4& res, int& count);

template <int MODE, int RATIO, int DT, int C, bool WIDE, int SMOOTH, bool REUSE, int NS,
          bool PACK>
__device__ __forceinline__ void march(const RenderArgs& a, const float4* s_lut, float* ring,
                                      const RaySeg& r, const Filt& F, float4& res,
                                      int& count) {
    using Smp = Sampler<DT, C, WIDE, REUSE, PACK, oob_reuse<MODE, DT, WIDE, REUSE>()>;
    const Smp smp(a.v);
    const int N = r.n;
    const float n_lut = (float)(a.lut_n - 1);
    res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    count = N;

    if (RATIO == 0) {
        GatherFeed<SMOOTH, NS, Smp> feed{smp, r, a.p.box_arm, ring, a.p};
        march_tf<MODE>(a, s_lut, r, F, feed, res, count);
        return;
    }
    {
        // Line ratio over two co-registered cubes (Section 4.5): method 1 keeps each cube's
        // maximum with strict '>' and maps max2/max1; method 2 maps the per-sample ratio
        // (DATAMIN -> 0 where cube 1 <= 0) and keeps its maximum with '>='.
        const Smp smp2(a.v2);
        const bool clip = a.p.filter == SVR_FILTER_CLIP;
        const float rinv = a.p.ratio_hi > a.p.ratio_lo ? 1.0f / (a.p.ratio_hi - a.p.ratio_lo) : 0.0f;
        float m1 = -INFINITY, m2 = -INFINITY, smax = -INFINITY;
        drive<3>(PairSource<Smp>(smp, smp2, r), N, [&](int, float2 v, bool active) -> bool {
            float v1 = v.x, v2 = v.y;
            if (clip) {
                v1 = (v1 < a.p.min_t || v1 > a.p.max_t) ? F.lo : v1;
                v2 = (v2 < a.p.min_t2 || v2 > a.p.max_t2) ? F.lo : v2;
            }
            if (RATIO == 1) {
                m1 = (active && v1 > m1) ? v1 : m1;
                m2 = (active && v2 > m2) ? v2 : m2;
            } else {
                const float s = v1 > 0.0f ? sat((v2 / v1 - a.p.ratio_lo) * rinv) : 0.0f;
                smax = (active && s >= smax) ? s : smax;
            }
            return active;
        });
        if (N > 0) {
            if (RATIO == 1) {
                if (m1 > 0.0f) {
                    res = table(s_lut, n_lut, sat((m2 / m1 - a.p.ratio_lo) * rinv));
                    if (a.p.mip_alpha == 1) res.w = 1.0f;
                }
            } else {
                res = table(s_lut, n_lut, smax);
                if (a.p.mip_alpha == 1) res.w = 1.0f;
            }
        }
    }
}

// setFragment of the MIP transfer functions (Alg. MIP0, MIP1, MIP_RGB) from the ray's maximum
// smax and the index kmax of its last maximal sample: MIP0 maps the maximum through the table,
// MIP1 colours by the location's velocity coordinate, MIP_RGB by its (z, y, x); alpha per
// mip_alpha (the Discussion's workaround for 2).
template <int MODE>
__device__ __forceinline__ float4 mip_fragment(const RenderArgs& a, const float4* s_lut,
                                               const RaySeg& r, const Filt& F, float smax,
                                               int kmax) {
    const float n_lut = (float)(a.lut_n - 1);
    float4 res;
    float alpha;
    if (MODE == SVR_MIP0) {
        res = table(s_lut, n_lut, smax);
        alpha = res.w;
    } else {
        const float km = (float)kmax;
        const float lx = sat((fmaf(km, r.step[0], r.p0[0]) + 0.5f) / (float)a.v.nx);
        const float ly = sat((fmaf(km, r.step[1], r.p0[1]) + 0.5f) / (float)a.v.ny);
        const float lz = sat((fmaf(km, r.step[2], r.p0[2]) + 0.5f) / (float)a.v.nz);
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
        const float sthr = F.inv > 0.0f ? sat((a.p.min_t - F.lo) * F.inv) : 0.0f;
        if (smax > sthr) alpha = 1.0f;
    }
    res.w = alpha;
    return res;
}

// Transfer functions of Sections 3.1-3.3 over the sample stream of one ray (any feed).
template <int MODE, class Feed>
__device__ __forceinline__ void march_tf(const RenderArgs& a, const float4* s_lut,
                                         const RaySeg& r, const Filt& F, Feed& feed,
                                         float4& res, int& count) {
    const int N = r.n;
    const float n_lut = (float)(a.lut_n - 1);
    res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    count = N;
    if (MODE <= SVR_MIPRGB) {
        // Eq. MIP, '>=' so a later sample wins a tie; MIP1/MIP_RGB keep the arg-max index.
        float smax = -INFINITY;
        int kmax = 0;
        feed.run([&](int k, float v, bool active) -> bool {
            const float s = F(v);
            if (MODE == SVR_MIP0) {
                smax = active ? fmaxf(s, smax) : smax;  // MIP0 keeps only the value
            } else {
                const bool take = active && s >= smax;
                smax = take ? s : smax;
                kmax = take ? k : kmax;
            }
            return active;
        });
        if (N == 0) return;
        res = mip_fragment<MODE>(a, s_lut, r, F, smax, kmax);
        return;
    }

    // Alg. AVIP0 / AVIP1 / AVIP_RGB: front-to-back compositing, stop after alpha > ert.
    const float kw = a.p.k, minv = a.p.min_val, ert = a.p.ert;
    const bool ofl = a.p.opacity_from_lut != 0;
    // normalised location of sample k per axis, loc = (p0 + k step + 0.5) / n, formed as one
    // clamped FMA from per-ray terms (within a few float32 roundings of the direct form)
    const float inx = 1.0f / (float)a.v.nx, iny = 1.0f / (float)a.v.ny, inz = 1.0f / (float)a.v.nz;
    const float lbx = (r.p0[0] + 0.5f) * inx, lsx = r.step[0] * inx;
    const float lby = (r.p0[1] + 0.5f) * iny, lsy = r.step[1] * iny;
    const float lbz = (r.p0[2] + 0.5f) * inz, lsz = r.step[2] * inz;
    Rgba t = {0.0f, 0.0f, 0.0f, 0.0f};
    int cnt = 0;
    feed.run([&](int k, float v, bool active) -> bool {
        const float s = F(v);
        const float kf = (float)k;
        float cr, cg, cb, op;
        if (MODE == SVR_AVIP0) {
            const float4 c = table(s_lut, n_lut, s);
            cr = c.x; cg = c.y; cb = c.z;
            op = ofl ? c.w : s;
        } else {
            const float lz = sat(fmaf(kf, lsz, lbz));
            if (MODE == SVR_AVIP1) {
                const float4 c = table(s_lut, n_lut, lz);
                cr = c.x; cg = c.y; cb = c.z;
            } else {
                cr = lz;
                cg = sat(fmaf(kf, lsy, lby));
                cb = sat(fmaf(kf, lsx, lbx));
            }
            op = ofl ? table(s_lut, n_lut, s).w : s;
        }
        const float al = composite(t, cr, cg, cb, op, kw, minv, active);
        cnt += active ? 1 : 0;
        return active && !(al > ert);
    });
    count = cnt;
    if (N > 0) res = make_float4(t.r, t.g, t.b, t.a);
}

// filter() of Alg. 1 and the colour-map domain for the launch's parameters.
__device__ __forceinline__ Filt make_filter(const RenderArgs& a) {
    Filt F;
    F.lo = a.p.clim_lo;
    float hi = a.p.clim_hi;
    if (!(hi > F.lo)) {
        F.lo = a.v.clim[0];
        hi = a.v.clim[1];
    }
    F.inv = hi > F.lo ? 1.0f / (hi - F.lo) : 0.0f;
    if (a.p.filter == SVR_FILTER_SCALE) {
        F.mn = a.p.min_t;
        F.mx = a.p.max_t;
        F.base = a.p.min_t;
        F.scale = a.p.max_t > a.p.min_t ? 1.0f / (a.p.max_t - a.p.min_t) : 0.0f;
    } else {
        F.mn = a.p.filter == SVR_FILTER_CLIP ? a.p.min_t : -INFINITY;
        F.mx = a.p.filter == SVR_FILTER_CLIP ? a.p.max_t : INFINITY;
        F.base = F.lo;
        F.scale = F.inv;
    }
    return F;
}

// The ray of pixel (px, py), or an empty one for lanes outside the image.
__device__ __forceinline__ RaySeg pixel_ray(const RenderArgs& a, int px, int py, bool inside) {
    RaySeg r;
    if (inside) {
        r = ray_segment(a.cam, px, py, a.v.nx, a.v.ny, a.v.nz, a.p.dt);
    } else {
        r.n = 0;
        r.q0[0] = r.q0[1] = r.q0[2] = 0.0;
        r.dq[0] = r.dq[1] = r.dq[2] = 0.0;
        r.p0[0] = r.p0[1] = r.p0[2] = 0.0f;
        r.step[0] = r.step[1] = r.step[2] = 0.0f;
    }
    return r;
}

// One ray of Alg. 1 for pixel (px, py).  Every lane of the wave calls this (the march loop
// is uniform); lanes outside the image pass inside = false and march no samples.  REUSE:
// same-cell corner reuse (float32 storage at steps below a voxel).  SMOOTH: the smoothing
// compiled in; the one-image kernels compile each kind into kernels of their own, so the
// plain march does not carry the registers of the box ring or the in-ray Gaussian.  NS:
// fetch slots of the sample loop.  PACK: 16-bit corners stay packed while in flight.
template <int MODE, int RATIO, int DT, int C, bool WIDE, bool REUSE = DT == SVR_F32,
          int SMOOTH = kSmoothAuto,
          int NS = drive_slots<MODE, DT, oob_reuse<MODE, DT, WIDE, REUSE>()>(), bool PACK = true>
__device__ __forceinline__ void render_ray(const RenderArgs& a, const float4* s_lut, float* ring,
                                           int px, int py, bool inside, float4& res,
                                           int& count) {
    const Filt F = make_filter(a);
    const RaySeg r = pixel_ray(a, px, py, inside);
    if constexpr (SMOOTH == kSmoothStar) {
        static_assert(RATIO == 0, "the in-ray Gaussian has no line-ratio form");
        march<MODE, 0, DT, C, WIDE, kSmoothStar, false, NS, PACK>(a, s_lut, ring, r, F, res, count);
    } else if constexpr (SMOOTH == kSmoothBox) {
        static_assert(RATIO == 0, "the line-ratio methods take no box smoothing");
        march<MODE, 0, DT, C, WIDE, kSmoothBox, REUSE, NS, PACK>(a, s_lut, ring, r, F, res, count);
    } else if constexpr (SMOOTH == kSmoothNone) {
        march<MODE, RATIO, DT, C, WIDE, kSmoothNone, REUSE, NS, PACK>(a, s_lut, ring, r, F, res, count);
    } else if (RATIO == 0 && a.p.box_arm > 0) {
        march<MODE, RATIO, DT, C, WIDE, kSmoothBox, REUSE, NS, PACK>(a, s_lut, ring, r, F, res, count);
    } else {
        march<MODE, RATIO, DT, C, WIDE, kSmoothNone, REUSE, NS, PACK>(a, s_lut, ring, r, F, res, count);
    }
}

// Pixel (lx, ly) of an 8x8 wave tile rendered by lane l.  The vector memory pipeline works
// on quarter-waves of 16 lanes and its cost grows with the distinct cache lines each quarter
// touches; for 4-byte voxels a 4x4 pixel block per quarter (Z order) touches fewer lines
// than an 8x2 strip, for 2-byte voxels (rows of half the length) the strip is cheaper.
template <int DT>
__device__ __forceinline__ void wave_pixel(int l, int& lx, int& ly) {
    if (DT == SVR_F32) {
        lx = (l & 1) | ((l >> 1) & 2) | ((l >> 2) & 4);
        ly = ((l >> 1) & 1) | ((l >> 2) & 2) | ((l >> 3) & 4);
    } else {
        lx = l & 7;
        ly = l >> 3;
    }
}

size_t render_lds_bytes(int lut_n, int box_arm, int ratio);

}  // namespace svr
