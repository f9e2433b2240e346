// Moment maps along the spectral axis (Section 2.2: the zeroth moment, Eq. mom0; the first
// moment, Eq. mom1; and the argmax variant).  A streaming reduction that reads every voxel of
// the channel window once: HBM-bound.
//
// One lane per spectrum (x, y).  The lanes of a wave take consecutive x, so each channel read
// is one contiguous row of 64 elements.  Each lane keeps 16 channel reads in flight ahead of
// their use.  The sums are float64, accumulated in channel order with every operation rounded
// separately, and rounded to float32 once at the end.
#include "common.h"

namespace svr {

constexpr int kMomAhead = 16;  // channel reads in flight per lane

struct MomAcc {
    double s0 = 0.0, s1 = 0.0;
    float best = 0.0f;
    int32_t arg = -1;
    // channel z with value v: counted when finite and inside [lo, hi]; ties in the maximum go
    // to the later channel (the MIP rule v_i >= c_{i-1})
    __device__ __forceinline__ void add(float v, int32_t z, float lo, float hi) {
#pragma clang fp contract(off)
        if (!(__builtin_isfinite(v) && v >= lo && v <= hi)) return;
        s0 = s0 + (double)v;
        s1 = s1 + (double)z * (double)v;
        if (arg < 0 || v >= best) {
            best = v;
            arg = z;
        }
    }
};

template <int DT>
__global__ __launch_bounds__(kBlock) void moments_kernel(const typename Elem<DT>::T* cube,
                                                         int32_t nx, int64_t sx, int64_t sy,
                                                         int64_t sz, int32_t z0, int32_t nzw,
                                                         double dv, float lo, float hi,
                                                         float* m0, float* m1, int32_t* amax) {
#pragma clang fp contract(off)
    const int x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y;
    const typename Elem<DT>::T* col = cube + (int64_t)y * sy + (int64_t)x * sx;
    MomAcc acc;
    const int32_t z1 = z0 + nzw;
    int32_t z = z0;
    for (; z + kMomAhead <= z1; z += kMomAhead) {
        float v[kMomAhead];
#pragma unroll
        for (int k = 0; k < kMomAhead; ++k) {
            const typename Elem<DT>::T e = load_nt(col + (int64_t)(z + k) * sz);
            v[k] = Elem<DT>::get(&e, 0);
        }
#pragma unroll
        for (int k = 0; k < kMomAhead; ++k) acc.add(v[k], z + k, lo, hi);
    }
    for (; z < z1; ++z) acc.add(Elem<DT>::get(col + (int64_t)z * sz, 0), z, lo, hi);
    const int64_t o = (int64_t)y * nx + x;
    if (m0) m0[o] = (float)(dv * acc.s0);
    if (m1) m1[o] = (acc.arg >= 0 && acc.s0 != 0.0) ? (float)(acc.s1 / acc.s0) : __builtin_nanf("");
    if (amax) amax[o] = acc.arg;
}

svr_status launch_moments(const svr_cube_view& c, int z0, int nzw, float dv, float lo, float hi,
                          float* m0, float* m1, int32_t* amax, hipStream_t stream) {
    const bool contig = c.sx == 0 && c.sy == 0 && c.sz == 0;
    const int64_t sx = contig ? 1 : c.sx;
    const int64_t sy = contig ? (int64_t)c.nx : c.sy;
    const int64_t sz = contig ? (int64_t)c.nx * c.ny : c.sz;
    const dim3 grid((unsigned)((c.nx + kBlock - 1) / kBlock), (unsigned)c.ny);
    const double dvd = (double)dv;
    switch (c.dtype) {
        case SVR_F16:
            hipLaunchKernelGGL(moments_kernel<SVR_F16>, grid, dim3(kBlock), 0, stream,
                               (const _Float16*)c.data, c.nx, sx, sy, sz, z0, nzw, dvd, lo, hi,
                               m0, m1, amax);
            break;
        case SVR_BF16:
            hipLaunchKernelGGL(moments_kernel<SVR_BF16>, grid, dim3(kBlock), 0, stream,
                               (const uint16_t*)c.data, c.nx, sx, sy, sz, z0, nzw, dvd, lo, hi,
                               m0, m1, amax);
            break;
        default:
            hipLaunchKernelGGL(moments_kernel<SVR_F32>, grid, dim3(kBlock), 0, stream,
                               (const float*)c.data, c.nx, sx, sy, sz, z0, nzw, dvd, lo, hi,
                               m0, m1, amax);
    }
    return hip_fail(hipGetLastError(), "moments launch");
}

}  // namespace svr
