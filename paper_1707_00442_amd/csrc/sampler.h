// Trilinear fetch from a bricked, aproned volume (clamp-to-edge), split into stages so the
// ray-march can issue the loads of a later sample before it blends the current one.
#pragma once

#include "common.h"

namespace svr {

// The 3D-texture fetch cube[loc] of Alg. 1 as trilinear interpolation: the point is
// clamped to [0, n-1] per axis, its cell (i, j, l) = floor(point) selects a brick and a
// local offset, and the eight corners are read at compile-time offsets from one address
// (the apron holds the +1 neighbours, so no corner leaves the brick and the upper edge
// needs no index clamp).  Interpolation order x, then y, then z, each a + f (b - a).
//
// WIDE = false addresses the storage with 32-bit byte offsets from a scalar base (volumes
// below 4 GiB); WIDE = true forms 64-bit addresses.
template <int DT, int C, bool WIDE>
struct Sampler {
    using T = typename Elem<DT>::T;
    static constexpr int E = C + 1;
    static constexpr int SH = C == 8 ? 3 : 4;
    static constexpr uint32_t kM24 = 0xffffffu;
    const T* data;
    float xm, ym, zm;
    uint32_t nbx, nby, pitch;

    // Loads in flight for one sample: its eight corners and the cell fractions.
    struct Fetch {
        float c000, c100, c010, c110, c001, c101, c011, c111;
        float fx, fy, fz;
    };

    // Brick counts and the pitch are below 2^24 (checked at volume creation); the masks
    // let the compiler use 24-bit multiplies.
    __device__ __forceinline__ explicit Sampler(const VolDesc& v)
        : data(static_cast<const T*>(v.data)),
          xm((float)(v.nx - 1)), ym((float)(v.ny - 1)), zm((float)(v.nz - 1)),
          nbx((uint32_t)v.nbx & kM24), nby((uint32_t)v.nby & kM24), pitch(v.pitch & kM24) {}

    // Element offset of voxel cell (ix, iy, iz) inside the bricked storage: brick index
    // (below 2^24) times the pitch plus the in-brick offset, below 2^32 in total.
    __device__ __forceinline__ uint32_t offset(uint32_t ix, uint32_t iy, uint32_t iz) const {
        __builtin_assume(ix <= kM24);
        __builtin_assume(iy <= kM24);
        __builtin_assume(iz <= kM24);
        uint32_t b = (iz >> SH) * nby + (iy >> SH);
        __builtin_assume(b <= kM24);
        b = b * nbx + (ix >> SH);
        __builtin_assume(b <= kM24);
        const uint32_t loc = ((iz & (C - 1)) * E + (iy & (C - 1))) * E + (ix & (C - 1));
        return b * pitch + loc;
    }

    __device__ __forceinline__ const T* at(uint32_t off) const {
        if (WIDE) return data + off;
        return reinterpret_cast<const T*>(reinterpret_cast<const char*>(data) +
                                          off * (uint32_t)sizeof(T));
    }

    // The point is clamped to [0, n-1], so the cell index is its truncation and the
    // fraction point - floor(point) is exact (v_fract).
    __device__ __forceinline__ Fetch fetch(float x, float y, float z) const {
        x = med3(x, 0.0f, xm);
        y = med3(y, 0.0f, ym);
        z = med3(z, 0.0f, zm);
        Fetch f;
        f.fx = __builtin_amdgcn_fractf(x);
        f.fy = __builtin_amdgcn_fractf(y);
        f.fz = __builtin_amdgcn_fractf(z);
        const T* q = at(offset((uint32_t)x, (uint32_t)y, (uint32_t)z));
        f.c000 = Elem<DT>::get(q, 0);
        f.c100 = Elem<DT>::get(q, 1);
        f.c010 = Elem<DT>::get(q, E);
        f.c110 = Elem<DT>::get(q, E + 1);
        f.c001 = Elem<DT>::get(q, E * E);
        f.c101 = Elem<DT>::get(q, E * E + 1);
        f.c011 = Elem<DT>::get(q, E * E + E);
        f.c111 = Elem<DT>::get(q, E * E + E + 1);
        return f;
    }

    static __device__ __forceinline__ float blend(const Fetch& f) {
        const float a00 = fmaf(f.fx, f.c100 - f.c000, f.c000);
        const float a10 = fmaf(f.fx, f.c110 - f.c010, f.c010);
        const float a01 = fmaf(f.fx, f.c101 - f.c001, f.c001);
        const float a11 = fmaf(f.fx, f.c111 - f.c011, f.c011);
        const float b0 = fmaf(f.fy, a10 - a00, a00);
        const float b1 = fmaf(f.fy, a11 - a01, a01);
        return fmaf(f.fz, b1 - b0, b0);
    }

    __device__ __forceinline__ float operator()(float x, float y, float z) const {
        return blend(fetch(x, y, z));
    }
};

// Samples along one ray: value j is the sample at p0 + (j + base) step.
template <class S>
struct RaySource {
    using Fetch = typename S::Fetch;
    const S& smp;
    float p0x, p0y, p0z, sx, sy, sz, base;
    __device__ __forceinline__ RaySource(const S& s, const RaySeg& r, float base_)
        : smp(s), p0x(r.p0[0]), p0y(r.p0[1]), p0z(r.p0[2]), sx(r.step[0]), sy(r.step[1]),
          sz(r.step[2]), base(base_) {}
    __device__ __forceinline__ Fetch fetch(float j) const {
        const float kf = j + base;
        return smp.fetch(fmaf(kf, sx, p0x), fmaf(kf, sy, p0y), fmaf(kf, sz, p0z));
    }
    static __device__ __forceinline__ float value(const Fetch& f) { return S::blend(f); }
};

// The same point sampled in two co-registered volumes (line ratios).
template <class S>
struct PairSource {
    struct Fetch {
        typename S::Fetch a, b;
    };
    RaySource<S> ra, rb;
    __device__ __forceinline__ PairSource(const S& s1, const S& s2, const RaySeg& r)
        : ra(s1, r, 0.0f), rb(s2, r, 0.0f) {}
    __device__ __forceinline__ Fetch fetch(float j) const { return Fetch{ra.fetch(j), rb.fetch(j)}; }
    static __device__ __forceinline__ float2 value(const Fetch& f) {
        return make_float2(S::blend(f.a), S::blend(f.b));
    }
};

// Drive alive = body(j, value_j, active) for j = 0, 1, 2, ... with the loads of the next two
// samples in flight while value j is blended.  The loop is unrolled three times with fixed
// roles for the three fetch slots (no slot is copied while its loads are outstanding) and
// its control is uniform across the wave: every lane runs every iteration, `active` tells a
// lane whether value j is one of its n samples and it is still alive, and the wave leaves
// once no lane needs a further sample.  Fetches of inactive lanes read clamped points
// inside the volume and are never used.
template <class Src, class Body>
__device__ __forceinline__ void drive(const Src& src, int n, Body&& body) {
    if (!wave_any(n > 0)) return;
    typename Src::Fetch q0 = src.fetch(0.0f);
    typename Src::Fetch q1 = src.fetch(1.0f);
    bool alive = true;
    float jf = 0.0f;
    for (int j = 0;; j += 3, jf += 3.0f) {
        typename Src::Fetch q2 = src.fetch(jf + 2.0f);
        alive = body(j, Src::value(q0), alive && j < n);
        q0 = src.fetch(jf + 3.0f);
        alive = body(j + 1, Src::value(q1), alive && j + 1 < n);
        q1 = src.fetch(jf + 4.0f);
        alive = body(j + 2, Src::value(q2), alive && j + 2 < n);
        if (!wave_any(alive && j + 3 < n)) break;
    }
}

}  // namespace svr
