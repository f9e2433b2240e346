// Trilinear fetch from a bricked, aproned volume (clamp-to-edge).
#pragma once

#include "common.h"

namespace svr {

// The 3D-texture fetch cube[loc] of Alg. 1 as trilinear interpolation: the point is
// clamped to [0, n-1] per axis, its cell (i, j, l) = floor(point) selects a brick and a
// local offset, and the eight corners are read at compile-time offsets from one address
// (the apron holds the +1 neighbours, so no corner leaves the brick and the upper edge
// needs no index clamp).  Interpolation order x, then y, then z, each a + f (b - a).
template <int DT, int C>
struct Sampler {
    using T = typename Elem<DT>::T;
    static constexpr int E = C + 1;
    static constexpr int SH = C == 8 ? 3 : 4;
    const T* data;
    float xm, ym, zm;
    uint32_t nbx, nby, pitch;

    __device__ __forceinline__ explicit Sampler(const VolDesc& v)
        : data(static_cast<const T*>(v.data)),
          xm((float)(v.nx - 1)), ym((float)(v.ny - 1)), zm((float)(v.nz - 1)),
          nbx((uint32_t)v.nbx), nby((uint32_t)v.nby), pitch(v.pitch) {}

    // Element offset of voxel cell (ix, iy, iz) inside the bricked storage.
    __device__ __forceinline__ uint32_t offset(uint32_t ix, uint32_t iy, uint32_t iz) const {
        const uint32_t b = ((iz >> SH) * nby + (iy >> SH)) * nbx + (ix >> SH);
        const uint32_t loc = ((iz & (C - 1)) * E + (iy & (C - 1))) * E + (ix & (C - 1));
        return b * pitch + loc;
    }

    __device__ __forceinline__ float operator()(float x, float y, float z) const {
        x = med3(x, 0.0f, xm);
        y = med3(y, 0.0f, ym);
        z = med3(z, 0.0f, zm);
        const float x0 = floorf(x), y0 = floorf(y), z0 = floorf(z);
        const float fx = x - x0, fy = y - y0, fz = z - z0;
        const T* q = data + offset((uint32_t)x0, (uint32_t)y0, (uint32_t)z0);
        const float c000 = Elem<DT>::get(q, 0);
        const float c100 = Elem<DT>::get(q, 1);
        const float c010 = Elem<DT>::get(q, E);
        const float c110 = Elem<DT>::get(q, E + 1);
        const float c001 = Elem<DT>::get(q, E * E);
        const float c101 = Elem<DT>::get(q, E * E + 1);
        const float c011 = Elem<DT>::get(q, E * E + E);
        const float c111 = Elem<DT>::get(q, E * E + E + 1);
        const float a00 = fmaf(fx, c100 - c000, c000);
        const float a10 = fmaf(fx, c110 - c010, c010);
        const float a01 = fmaf(fx, c101 - c001, c001);
        const float a11 = fmaf(fx, c111 - c011, c011);
        const float b0 = fmaf(fy, a10 - a00, a00);
        const float b1 = fmaf(fy, a11 - a01, a01);
        return fmaf(fz, b1 - b0, b0);
    }
};

}  // namespace svr
