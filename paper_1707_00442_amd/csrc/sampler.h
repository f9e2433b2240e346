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
// Float32 storage reads the corners as four (x, x + 1) pairs; 16-bit storage (y-pair
// layout) as two runs of four elements, the faces z and z + 1 of the cell.
//
// WIDE = false addresses the storage with 32-bit byte offsets from a scalar base (volumes
// below 4 GiB); WIDE = true forms 64-bit addresses.  REUSE enables the same-cell reuse of
// RaySource (float32 storage only).  PACK keeps 16-bit corners packed while their loads are
// in flight (see Fetch).  OOB makes reuse issue the loads of a repeated cell too, out of the
// buffer's range (see fetch_after).
template <int DT, int C, bool WIDE, bool REUSE = DT == SVR_F32, bool PACK = true,
          bool OOB = false>
struct Sampler {
    using T = typename Elem<DT>::T;
    static constexpr int E = C + 1;
    static constexpr int SH = C == 8 ? 3 : 4;
    static constexpr uint32_t kM24 = 0xffffffu;
    // Same-cell reuse pays for float32 storage (four 8-byte loads per sample) at steps below
    // a voxel; with two loads per sample (16-bit storage), or at steps where every sample
    // changes cell, its selects and registers cost more than it saves.
    static constexpr bool kReuse = REUSE && DT == SVR_F32;
    static constexpr bool kPack = PACK && DT != SVR_F32;
    static constexpr bool kOob = OOB && kReuse && !WIDE;
    const T* data;
    double xm, ym, zm;
    uint32_t nbx, nby, pitch;
    __amdgpu_buffer_rsrc_t rsrc;  // the whole storage as one buffer (used by kOob)

    // Loads in flight for one sample: its eight corners and the cell fractions; reuse marks
    // a sample in the same cell as the one fetched before it (no loads issued, corners 0).
    // Packed 16-bit fetches keep the four loaded words (two corners each) and convert them
    // only when the sample is blended, so a fetch slot holds half the registers while in
    // flight; that lets the render kernels keep more samples in flight at the same occupancy.
    struct FetchF32 {
        float c000, c100, c010, c110, c001, c101, c011, c111;
        float fx, fy, fz;
        bool reuse;
    };
    struct FetchPacked {
        uint32_t w0, w1, w2, w3;  // (c000, c010), (c100, c110), (c001, c011), (c101, c111)
        float fx, fy, fz;
        bool reuse;
    };
    using Fetch = typename std::conditional<kPack, FetchPacked, FetchF32>::type;

    // Brick counts and the pitch are below 2^24 (checked at volume creation); the masks
    // let the compiler use 24-bit multiplies.
    __device__ __forceinline__ explicit Sampler(const VolDesc& v)
        : data(static_cast<const T*>(v.data)),
          xm((double)(v.nx - 1)), ym((double)(v.ny - 1)), zm((double)(v.nz - 1)),
          nbx((uint32_t)v.nbx & kM24), nby((uint32_t)v.nby & kM24), pitch(v.pitch & kM24),
          rsrc(__builtin_amdgcn_make_buffer_rsrc(
              const_cast<void*>(v.data), (short)0,
              (int)(uint32_t)((uint64_t)v.nbx * v.nby * v.nbz * v.pitch * sizeof(T)),
              kBufferDword3)) {}

    // Buffer descriptor word 3: 32-bit data format (raw loads), range checking on.
    static constexpr int kBufferDword3 = 0x00020000;

    // Element offset of voxel cell (ix, iy, iz) inside the bricked storage: brick index
    // (below 2^24) times the pitch plus the in-brick offset, below 2^32 in total.
    __device__ __forceinline__ uint32_t offset(uint32_t ix, uint32_t iy, uint32_t iz) const {
        return cell_offset<DT, C>(ix, iy, iz, nbx, nby, pitch);
    }

    __device__ __forceinline__ const T* at(uint32_t off) const {
        if (WIDE) return data + off;
        return reinterpret_cast<const T*>(reinterpret_cast<const char*>(data) +
                                          off * (uint32_t)sizeof(T));
    }

    // The point (double) is clamped to [0, n-1], so the cell index is its truncation; the
    // fraction point - floor(point) is exact in double (v_fract) and then rounded to float.
    __device__ __forceinline__ Fetch fetch(double x, double y, double z) const {
        uint32_t none = 0xffffffffu;
        return fetch_after(x, y, z, none);
    }

    // As fetch(), but the loads are skipped when the cell is the one at element offset
    // `last` (the previous sample's); `last` becomes this sample's cell.  Offsets are below
    // 2^32 - 1, so 0xffffffff matches no cell.
    __device__ __forceinline__ Fetch fetch_after(double x, double y, double z,
                                                 uint32_t& last) const {
        x = fmin(fmax(x, 0.0), xm);
        y = fmin(fmax(y, 0.0), ym);
        z = fmin(fmax(z, 0.0), zm);
        Fetch f;
        f.fx = (float)__builtin_amdgcn_fract(x);
        f.fy = (float)__builtin_amdgcn_fract(y);
        f.fz = (float)__builtin_amdgcn_fract(z);
        const uint32_t o = offset((uint32_t)x, (uint32_t)y, (uint32_t)z);
        f.reuse = kReuse && o == last;
        last = o;
        if constexpr (kOob) {
            // Reuse without a branch: a repeated cell's loads are issued at an offset past
            // the end of any 32-bit addressed storage (such storage ends below kPastStorage,
            // larger volumes take the 64-bit path), where buffer loads return 0 without
            // touching memory.  Every sample then issues the same four loads, so the loads
            // of later samples stay in flight while this one is blended (behind a branch the
            // waits before each blend must assume none were issued).
            constexpr uint32_t kPast = kPastStorage;
            const uint32_t b = f.reuse ? kPast : o * 4u;
            const auto p0 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, b, 0, 0);
            const auto p1 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, b + 4u * E, 0, 0);
            const auto p2 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, b + 4u * E * E, 0, 0);
            const auto p3 = __builtin_amdgcn_raw_buffer_load_b64(rsrc, b + 4u * (E * E + E), 0, 0);
            f.c000 = __uint_as_float(p0[0]);
            f.c100 = __uint_as_float(p0[1]);
            f.c010 = __uint_as_float(p1[0]);
            f.c110 = __uint_as_float(p1[1]);
            f.c001 = __uint_as_float(p2[0]);
            f.c101 = __uint_as_float(p2[1]);
            f.c011 = __uint_as_float(p3[0]);
            f.c111 = __uint_as_float(p3[1]);
            return f;
        }
        if constexpr (!kPack) {
            if (f.reuse) {
                f.c000 = f.c100 = f.c010 = f.c110 = f.c001 = f.c101 = f.c011 = f.c111 = 0.0f;
                return f;
            }
        }
        const T* q = at(o);
        if constexpr (DT == SVR_F32) {
            f.c000 = Elem<DT>::get(q, 0);
            f.c100 = Elem<DT>::get(q, 1);
            f.c010 = Elem<DT>::get(q, E);
            f.c110 = Elem<DT>::get(q, E + 1);
            f.c001 = Elem<DT>::get(q, E * E);
            f.c101 = Elem<DT>::get(q, E * E + 1);
            f.c011 = Elem<DT>::get(q, E * E + E);
            f.c111 = Elem<DT>::get(q, E * E + E + 1);
        } else if constexpr (!kPack) {
            constexpr uint32_t kZ = 2 * C * E;  // next pair layer
            f.c000 = Elem<DT>::get(q, 0);
            f.c010 = Elem<DT>::get(q, 1);
            f.c100 = Elem<DT>::get(q, 2);
            f.c110 = Elem<DT>::get(q, 3);
            f.c001 = Elem<DT>::get(q, kZ);
            f.c011 = Elem<DT>::get(q, kZ + 1);
            f.c101 = Elem<DT>::get(q, kZ + 2);
            f.c111 = Elem<DT>::get(q, kZ + 3);
        } else {
            // pair elements start at even element offsets, so each pair is one aligned word
            constexpr uint32_t kZw = C * E;  // next pair layer, in 32-bit words
            const uint32_t* qw = reinterpret_cast<const uint32_t*>(q);
            f.w0 = qw[0];
            f.w1 = qw[1];
            f.w2 = qw[kZw];
            f.w3 = qw[kZw + 1];
        }
        return f;
    }

    // element h (0 = low, 1 = high half) of a word of two 16-bit elements, as float
    static __device__ __forceinline__ float half(uint32_t w, int h) {
        if constexpr (DT == SVR_BF16) return __uint_as_float(h ? (w & 0xffff0000u) : (w << 16));
        else return (float)__builtin_bit_cast(_Float16, (uint16_t)(h ? (w >> 16) : w));
    }

    static __device__ __forceinline__ float blend(const Fetch& f) {
        float c000, c100, c010, c110, c001, c101, c011, c111;
        if constexpr (!kPack) {
            c000 = f.c000; c100 = f.c100; c010 = f.c010; c110 = f.c110;
            c001 = f.c001; c101 = f.c101; c011 = f.c011; c111 = f.c111;
        } else {
            c000 = half(f.w0, 0); c010 = half(f.w0, 1); c100 = half(f.w1, 0); c110 = half(f.w1, 1);
            c001 = half(f.w2, 0); c011 = half(f.w2, 1); c101 = half(f.w3, 0); c111 = half(f.w3, 1);
        }
        const float a00 = fmaf(f.fx, c100 - c000, c000);
        const float a10 = fmaf(f.fx, c110 - c010, c010);
        const float a01 = fmaf(f.fx, c101 - c001, c001);
        const float a11 = fmaf(f.fx, c111 - c011, c011);
        const float b0 = fmaf(f.fy, a10 - a00, a00);
        const float b1 = fmaf(f.fy, a11 - a01, a01);
        return fmaf(f.fz, b1 - b0, b0);
    }

    __device__ __forceinline__ float operator()(double x, double y, double z) const {
        return blend(fetch(x, y, z));
    }
};

// Samples along one ray, fetched in order: fetch number j (j = 0, 1, 2, ...) is the sample
// at q0 + (j + base) dq, each position formed directly in double (one fma per axis from the
// sample index), so a sample's position does not depend on where the stream started: a ray
// rendered in segments (split MIP rays) samples exactly the points of the whole ray.  At
// steps below a voxel consecutive samples often share a cell: such a sample issues no loads
// and value() blends it from the corners of the last sample that loaded (values are taken in
// fetch order, so those are the previous sample's corners).
template <class S>
struct RaySource {
    using Fetch = typename S::Fetch;
    const S& smp;
    double qx, qy, qz, dqx, dqy, dqz, kd;
    uint32_t last = 0xffffffffu;
    Fetch lc{};  // corners of the last blended sample that loaded
    __device__ __forceinline__ RaySource(const S& s, const RaySeg& r, float base)
        : smp(s), qx(r.q0[0]), qy(r.q0[1]), qz(r.q0[2]), dqx(r.dq[0]), dqy(r.dq[1]),
          dqz(r.dq[2]), kd((double)base) {}
    __device__ __forceinline__ Fetch next() {
        const Fetch f = smp.fetch_after(fma(kd, dqx, qx), fma(kd, dqy, qy), fma(kd, dqz, qz),
                                        last);
        kd += 1.0;
        return f;
    }
    __device__ __forceinline__ float value(const Fetch& f) {
        if constexpr (!S::kReuse) {
            return S::blend(f);
        } else {
            const bool r = f.reuse;
            lc.c000 = r ? lc.c000 : f.c000;
            lc.c100 = r ? lc.c100 : f.c100;
            lc.c010 = r ? lc.c010 : f.c010;
            lc.c110 = r ? lc.c110 : f.c110;
            lc.c001 = r ? lc.c001 : f.c001;
            lc.c101 = r ? lc.c101 : f.c101;
            lc.c011 = r ? lc.c011 : f.c011;
            lc.c111 = r ? lc.c111 : f.c111;
            lc.fx = f.fx;
            lc.fy = f.fy;
            lc.fz = f.fz;
            return S::blend(lc);
        }
    }
};

// The in-ray 3-axis Gaussian of Section 4.2 (Alg. 9-tap smoothing, applied to the data axes
// in turn): a sample value v at point p becomes, for e = x, then y, then z,
// v <- c0 v + sum_k w_k (cube[p + off_k e] + cube[p - off_k e]), every lookup a trilinear
// fetch of the raw cube.  The six fetches of one offset pair are independent and issued
// together; the value is complete when next() returns.  The taps are read from the launch
// parameters (svr_params star_n, star_c0, star_off, star_w).
template <class S>
struct StarSource {
    using Fetch = float;
    const S& smp;
    const svr_params& st;
    double px, py, pz, dqx, dqy, dqz;
    __device__ __forceinline__ StarSource(const S& s, const svr_params& t, const RaySeg& r)
        : smp(s), st(t), px(r.q0[0]), py(r.q0[1]), pz(r.q0[2]), dqx(r.dq[0]), dqy(r.dq[1]),
          dqz(r.dq[2]) {}
    __device__ __forceinline__ float star(double x, double y, double z) const {
        float v = smp(x, y, z);
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;  // per-axis sums over the pairs, in order
        for (int k = 0; k < st.star_n; ++k) {
            const double o = (double)st.star_off[k];
            const float w = st.star_w[k];
            const float xp = smp(x + o, y, z), xm = smp(x - o, y, z);
            const float yp = smp(x, y + o, z), ym = smp(x, y - o, z);
            const float zp = smp(x, y, z + o), zm = smp(x, y, z - o);
            sx = fmaf(xm, w, fmaf(xp, w, sx));
            sy = fmaf(ym, w, fmaf(yp, w, sy));
            sz = fmaf(zm, w, fmaf(zp, w, sz));
        }
        v = fmaf(v, st.star_c0, sx);
        v = fmaf(v, st.star_c0, sy);
        return fmaf(v, st.star_c0, sz);
    }
    __device__ __forceinline__ Fetch next() {
        const float v = star(px, py, pz);
        px += dqx;
        py += dqy;
        pz += dqz;
        return v;
    }
    __device__ __forceinline__ float value(const Fetch& f) const { return f; }
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
    __device__ __forceinline__ Fetch next() { return Fetch{ra.next(), rb.next()}; }
    __device__ __forceinline__ float2 value(const Fetch& f) {
        const float va = ra.value(f.a);
        return make_float2(va, rb.value(f.b));
    }
};

// Drive alive = body(j, value_j, active) for j = 0, 1, 2, ... with the loads of the next
// NS - 1 samples in flight while value j is blended.  The loop is unrolled NS times with
// fixed roles for the NS fetch slots (no slot is copied while its loads are outstanding) and
// its control is uniform across the wave: every lane runs every iteration, `active` tells a
// lane whether value j is one of its n samples and it is still alive, and the wave leaves
// once no lane needs a further sample.  Fetches of inactive lanes read clamped points
// inside the volume and are never used.
template <int NS, class Src, class Body>
__device__ __forceinline__ void drive(Src src, int n, Body&& body) {
    static_assert(NS >= 2, "at least one sample in flight");
    if (!wave_any(n > 0)) return;
    typename Src::Fetch q[NS];
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) q[s] = src.next();
    bool alive = true;
    for (int j = 0;; j += NS) {
        q[NS - 1] = src.next();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            alive = body(j + s, src.value(q[s]), alive && j + s < n);
            if (s < NS - 1) q[s] = src.next();
        }
        if (!wave_any(alive && j + NS < n)) break;
    }
}

// Same-cell reuse through out-of-range loads (Sampler, OOB) for float32 storage addressed
// with 32-bit offsets: measured faster for the AVIP transfer functions (AVIP0 at 8 slots
// 10% faster, AVIP1 at 9 slots 7%, AVIP_RGB 2%), slower for MIP1 and MIP_RGB (5-10%).
// MIP0 gains on large volumes (the split renders use it, below) but lost 20% on a
// cache-resident 64^3 cube, where every load costs texture-path time and none waits on HBM.
template <int MODE, int DT, bool WIDE, bool REUSE>
constexpr bool oob_reuse() {
    return REUSE && !WIDE && DT == SVR_F32 &&
           (MODE == SVR_AVIP0 || MODE == SVR_AVIP1 || MODE == SVR_AVIPRGB);
}
// The split MIP renders (large oblique views) take the out-of-range loads too: MIP0 always,
// MIP1 and MIP_RGB without box smoothing, where their launches are capped at two workgroups
// per CU (uncapped, at 128 VGPRs, they ran four waves per SIMD and were slower than with
// the reuse branch).
template <int MODE, int DT, bool WIDE, bool REUSE, bool BOX>
constexpr bool oob_reuse_split() {
    return oob_reuse<MODE, DT, WIDE, REUSE>() ||
           (REUSE && !WIDE && DT == SVR_F32 &&
            (MODE == SVR_MIP0 || (MODE <= SVR_MIPRGB && !BOX)));
}

// Fetch slots of the sample loop per transfer function and storage type (measured on the
// 512 x 512 x 1024 rotation views: deeper pipelines keep more loads in flight per wave but
// need more registers, so the best depth depends on the per-sample state each mode keeps;
// packed 16-bit slots are half the size of float32 ones and go deeper).
template <int MODE, int DT, bool OOB = false>
constexpr int drive_slots() {
    // split MIP1 / MIP_RGB with the reuse loads, two waves per SIMD: 8 slots 2.41 ms, 6 2.51,
    // 5 2.61, 10 2.44, 12 2.42
    if ((MODE == SVR_MIP1 || MODE == SVR_MIPRGB) && DT == SVR_F32 && OOB) return 8;
    if (MODE == SVR_MIP0 || MODE == SVR_MIP1 || MODE == SVR_MIPRGB) return DT == SVR_F32 ? 6 : 8;
    if (MODE == SVR_AVIPRGB) return DT == SVR_F32 ? 5 : 7;
    if (MODE == SVR_AVIP0) return OOB ? 8 : 6;
    return DT == SVR_F32 ? (OOB ? 9 : 7) : 8;  // SVR_AVIP1
}

}  // namespace svr
