// Forward ray-march (Alg. 1 with the transfer functions of Section 3, the box smoothing of
// Section 4.1, the filters of Sections 4.3/4.4 and the line-ratio methods of Section 4.5).
//
// One lane per ray.  A 256-lane workgroup covers a 16x16 pixel tile as four 8x8 wave tiles;
// tiles are dealt to XCDs in contiguous runs.  Ray setup is FP64 (once per ray); the hot
// loop is FP32: a trilinear fetch from the bricked, aproned volume (eight loads sharing one
// address), the filter, the transfer function and compositing.  The colour table and the
// per-lane box-smoothing ring live in LDS.  The sample loop is uniform across the wave, with
// the loads of further samples in flight while a sample is blended; the wave leaves it
// once none of its rays needs another sample (AVIP early termination is per ray).
#include "march.h"

namespace svr {

template <int MODE, int RATIO, int DT, int C, bool WIDE, bool REUSE, int SMOOTH>
__global__ __launch_bounds__(kBlock) void render_kernel(const RenderArgs a) {
    extern __shared__ float4 smem[];
    float4* s_lut = smem;
    const int n_lut = a.lut_n;
    stage_table(s_lut, a.lut, n_lut);
    __syncthreads();

    const int t = xcd_tile((int)blockIdx.x, a.nblocks);
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int lx, ly;
    wave_pixel<DT>(l, lx, ly);
    const int px = tx * kTile + (w & 1) * 8 + lx;
    const int py = ty * kTile + (w >> 1) * 8 + ly;
    const bool inside = px < a.cam.width && py < a.cam.height;

    float4 res;
    int count;
    float* ring = reinterpret_cast<float*>(smem + n_lut + 1) + threadIdx.x;
    render_ray<MODE, RATIO, DT, C, WIDE, REUSE, SMOOTH>(a, s_lut, ring, px, py, inside, res,
                                                        count);
    if (inside) {
        const size_t pix = (size_t)py * a.cam.width + px;
        a.out[pix] = res;
        if (a.samples) a.samples[pix] = count;
    }
}

using RenderFn = void (*)(RenderArgs);

// The kernel for one transfer function (or line-ratio method) and smoothing kind.  The
// line-ratio methods exist only without smoothing (the parameter checks reject the rest).
template <int DT, int C, bool WIDE, bool REUSE, int SMOOTH>
static RenderFn pick(int mode, int ratio) {
    if constexpr (SMOOTH == kSmoothNone || SMOOTH == kSmoothAuto) {
        if (ratio == 1) return render_kernel<SVR_MIP0, 1, DT, C, WIDE, REUSE, SMOOTH>;
        if (ratio == 2) return render_kernel<SVR_MIP0, 2, DT, C, WIDE, REUSE, SMOOTH>;
    }
    switch (mode) {
        case SVR_MIP0: return render_kernel<SVR_MIP0, 0, DT, C, WIDE, REUSE, SMOOTH>;
        case SVR_MIP1: return render_kernel<SVR_MIP1, 0, DT, C, WIDE, REUSE, SMOOTH>;
        case SVR_MIPRGB: return render_kernel<SVR_MIPRGB, 0, DT, C, WIDE, REUSE, SMOOTH>;
        case SVR_AVIP0: return render_kernel<SVR_AVIP0, 0, DT, C, WIDE, REUSE, SMOOTH>;
        case SVR_AVIP1: return render_kernel<SVR_AVIP1, 0, DT, C, WIDE, REUSE, SMOOTH>;
        default: return render_kernel<SVR_AVIPRGB, 0, DT, C, WIDE, REUSE, SMOOTH>;
    }
}

template <int DT, int C, bool WIDE, bool REUSE>
static RenderFn pick_smooth(int smooth, int mode, int ratio) {
    if (smooth == kSmoothBox) return pick<DT, C, WIDE, REUSE, kSmoothBox>(mode, ratio);
    return pick<DT, C, WIDE, REUSE, kSmoothNone>(mode, ratio);
}

template <int C, bool WIDE>
static RenderFn pick_dt(int dtype, bool reuse, int smooth, int mode, int ratio) {
    // In-ray Gaussian kernels: no reuse, the stencil's fetches are not along the ray.
    if (smooth == kSmoothStar) {
        if (dtype == SVR_F16) return pick<SVR_F16, C, WIDE, false, kSmoothStar>(mode, 0);
        if (dtype == SVR_BF16) return pick<SVR_BF16, C, WIDE, false, kSmoothStar>(mode, 0);
        return pick<SVR_F32, C, WIDE, false, kSmoothStar>(mode, 0);
    }
    if (dtype == SVR_F16) return pick_smooth<SVR_F16, C, WIDE, false>(smooth, mode, ratio);
    if (dtype == SVR_BF16) return pick_smooth<SVR_BF16, C, WIDE, false>(smooth, mode, ratio);
    // Float32 without reuse keeps the plain and box marches in one kernel: compiled alone,
    // the plain MIP march had its loads sunk to their uses (no sample in flight) and the
    // one-sample-per-voxel views ran 2.5x slower.
    return reuse ? pick_smooth<SVR_F32, C, WIDE, true>(smooth, mode, ratio)
                 : pick<SVR_F32, C, WIDE, false, kSmoothAuto>(mode, ratio);
}

// Same-cell reuse (float32 storage) only where consecutive samples can share a cell: steps
// below one voxel.
static RenderFn pick_any(int dtype, int brick, bool wide, float dt, int smooth, int mode,
                         int ratio) {
    const bool reuse = dtype == SVR_F32 && dt < 1.0f;
    if (brick == 16)
        return wide ? pick_dt<16, true>(dtype, reuse, smooth, mode, ratio)
                    : pick_dt<16, false>(dtype, reuse, smooth, mode, ratio);
    return wide ? pick_dt<8, true>(dtype, reuse, smooth, mode, ratio)
                : pick_dt<8, false>(dtype, reuse, smooth, mode, ratio);
}

size_t render_lds_bytes(int lut_n, int box_arm, int ratio) {
    size_t b = (size_t)(lut_n + 1) * sizeof(float4);
    if (ratio == 0 && box_arm > 0) b += (size_t)(2 * box_arm + 1) * kBlock * sizeof(float);
    return b;
}

svr_status launch_render(const svr_volume* v, const svr_volume* v2, const svr_camera& cam,
                         const svr_lut& lut, const svr_params& p, float* out,
                         int32_t* samples, hipStream_t stream) {
    RenderArgs a;
    a.v = v->d;
    a.v2 = v2 ? v2->d : v->d;
    a.cam = cam;
    a.lut = reinterpret_cast<const float4*>(lut.rgba);
    a.lut_n = lut.n;
    a.p = p;
    a.out = reinterpret_cast<float4*>(out);
    a.samples = samples;
    a.tiles_x = (cam.width + kTile - 1) / kTile;
    const int tiles_y = (cam.height + kTile - 1) / kTile;
    a.nblocks = a.tiles_x * tiles_y;
    const bool wide = wide_volume(v->d) || (v2 != nullptr && wide_volume(v2->d));
    const int smooth = p.star_n > 0 ? kSmoothStar
                       : (p.ratio == 0 && p.box_arm > 0) ? kSmoothBox : kSmoothNone;
    RenderFn fn = pick_any(v->d.dtype, v->d.brick, wide, p.dt, smooth, p.mode, p.ratio);
    const size_t lds = render_lds_bytes(lut.n, p.box_arm, p.ratio);
    hipLaunchKernelGGL(fn, dim3(a.nblocks), dim3(kBlock), lds, stream, a);
    return hip_fail(hipGetLastError(), "render launch");
}

}  // namespace svr
