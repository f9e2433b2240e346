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

    const int t = xcd_run_tile((int)blockIdx.x, a.nblocks);
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

// ------------------------------------------------------------------ split MIP rays
// Oblique views with few rays leave the SIMDs short of waves to hide the latency of their
// gathers.  For the MIP transfer functions the samples of a ray can be split into nseg
// segments rendered by different workgroups: each segment keeps its maximum s and the index
// k of its last maximal sample, and the per-pixel maximum of the 64-bit keys (s << 32 | k),
// larger s first, then the later k, is Eq. MIP's '>=' over the whole ray exactly.  Sample
// positions are formed from the sample index (RaySource) and a box-smoothed segment starts
// its raw stream box_arm samples early, so every segment sees the values of the whole ray
// and the image equals the one-pass render.  The key lives in the first 8 bytes of the
// pixel's output until the finalising kernel writes the fragment there.

// Unsigned integers ordered as the floats they encode (-0 taken as +0): the sign bit is set
// for non-negative values and every bit is inverted for negative ones.
__device__ __forceinline__ uint32_t order_key(float x) {
    const uint32_t u = __float_as_uint(x + 0.0f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float order_value(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void split_clear_kernel(unsigned long long* key, int64_t npix) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npix) key[2 * i] = 0ull;
}

template <int MODE, int DT, int C, bool WIDE, bool REUSE, int SMOOTH>
__global__ __launch_bounds__(kBlock) void render_split_kernel(const RenderArgs a, int32_t nseg) {
    extern __shared__ float4 smem[];  // the box ring (SMOOTH = kSmoothBox)
    const int tiles = a.nblocks;
    const int b = (int)blockIdx.x;
    const int seg = b / tiles;
    const int t = xcd_run_tile(b - seg * tiles, tiles);
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int lx, ly;
    wave_pixel<DT>(l, lx, ly);
    const int px = tx * kTile + (w & 1) * 8 + lx;
    const int py = ty * kTile + (w >> 1) * 8 + ly;
    const bool inside = px < a.cam.width && py < a.cam.height;
    const Filt F = make_filter(a);
    RaySeg r = pixel_ray(a, px, py, inside);
    const int len = (r.n + nseg - 1) / nseg;
    const int k0 = seg * len;
    const int n = max(min(len, r.n - k0), 0);
    constexpr bool OOB = oob_reuse_split<MODE, DT, WIDE, REUSE, SMOOTH == kSmoothBox>();
    using Smp = Sampler<DT, C, WIDE, REUSE, true, OOB>;
    const Smp smp(a.v);
    float smax = -INFINITY;
    int kmax = 0;
    float* ring = reinterpret_cast<float*>(smem) + threadIdx.x;
    for_each_value_from<SMOOTH, drive_slots<MODE, DT, OOB>()>(smp, r, k0, n, a.p.box_arm, ring,
                                   [&](int k, float v, bool active) -> bool {
                                       const float s = F(v);
                                       if (MODE == SVR_MIP0) {
                                           smax = active ? fmaxf(s, smax) : smax;
                                       } else {
                                           const bool take = active && s >= smax;
                                           smax = take ? s : smax;
                                           kmax = take ? k : kmax;
                                       }
                                       return active;
                                   });
    if (inside && n > 0) {
        const unsigned long long key =
            ((unsigned long long)order_key(smax) << 32) | (unsigned long long)(uint32_t)(k0 + kmax);
        atomicMax(reinterpret_cast<unsigned long long*>(a.out) +
                      2 * ((size_t)py * a.cam.width + px),
                  key);
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void split_finalize_kernel(const RenderArgs a) {
    extern __shared__ float4 smem[];
    float4* s_lut = smem;
    stage_table(s_lut, a.lut, a.lut_n);
    __syncthreads();
    const int t = xcd_run_tile((int)blockIdx.x, a.nblocks);
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const int px = tx * kTile + (threadIdx.x & 15);
    const int py = ty * kTile + (threadIdx.x >> 4);
    if (px >= a.cam.width || py >= a.cam.height) return;
    const Filt F = make_filter(a);
    const RaySeg r = pixel_ray(a, px, py, true);
    const size_t pix = (size_t)py * a.cam.width + px;
    float4 res = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (r.n > 0) {
        const unsigned long long key = reinterpret_cast<const unsigned long long*>(a.out)[2 * pix];
        res = mip_fragment<MODE>(a, s_lut, r, F, order_value((uint32_t)(key >> 32)),
                                 (int)(uint32_t)key);
    }
    a.out[pix] = res;
    if (a.samples) a.samples[pix] = r.n;
}

using SplitFn = void (*)(RenderArgs, int32_t);

template <int DT, int C, bool WIDE, bool REUSE, int SMOOTH>
static SplitFn pick_split_mode(int mode) {
    if (mode == SVR_MIP0) return render_split_kernel<SVR_MIP0, DT, C, WIDE, REUSE, SMOOTH>;
    if (mode == SVR_MIP1) return render_split_kernel<SVR_MIP1, DT, C, WIDE, REUSE, SMOOTH>;
    return render_split_kernel<SVR_MIPRGB, DT, C, WIDE, REUSE, SMOOTH>;
}

template <int DT, int C, bool WIDE, bool REUSE>
static SplitFn pick_split(int mode, bool box) {
    return box ? pick_split_mode<DT, C, WIDE, REUSE, kSmoothBox>(mode)
               : pick_split_mode<DT, C, WIDE, REUSE, kSmoothNone>(mode);
}

// The split kernel for a volume's storage type, brick edge and addressing (REUSE as the
// one-pass path: float32 storage at steps below a voxel).
static SplitFn pick_split_any(int dtype, int brick, bool wide, float dt, int mode, bool box) {
    const bool reuse = dtype == SVR_F32 && dt < 1.0f;
#define SVR_SPLIT_DT(C, W)                                                                 \
    if (dtype == SVR_F16) return pick_split<SVR_F16, C, W, false>(mode, box);             \
    if (dtype == SVR_BF16) return pick_split<SVR_BF16, C, W, false>(mode, box);           \
    return reuse ? pick_split<SVR_F32, C, W, true>(mode, box)                              \
                 : pick_split<SVR_F32, C, W, false>(mode, box)
    if (brick == 16) {
        if (wide) { SVR_SPLIT_DT(16, true); }
        SVR_SPLIT_DT(16, false);
    }
    if (wide) { SVR_SPLIT_DT(8, true); }
    SVR_SPLIT_DT(8, false);
#undef SVR_SPLIT_DT
}

// Segments per ray for a MIP render.  Oblique views are bound by the latency of their
// scattered corner gathers, so they gain from more rays in flight: measured on the
// 512 x 512 x 1024 cube at dt = 0.5, a 256 x 256 view ran 1.33x faster in 8 segments and the
// 1920 x 1080 views 6% faster in 2; a 512 x 512 view was unchanged.  The target is about
// 2^21 ray segments (8 ray waves per SIMD, in about two rounds at the MIP kernels' two waves
// per SIMD), at most 8 segments, each of at least 256 samples on the longest ray: each
// segment repeats the ray setup and fills and drains the fetch pipeline, and 1000 x 1000
// views of a 128^3 cube (rays of up to 222 samples) ran 13% slower in 3 segments.  Parallel
// views along a volume axis are excluded: their quarter-waves read whole cache lines in
// brick order, one pass already streams at the HBM limit, and split into 2-8 concurrent
// streams the low-density view ran 1.3-1.6x slower.  Below about 2^24 samples a render is
// launch-bound and stays one pass.
static bool axis_parallel(const svr_camera& cam) {
    if (cam.type != 0) return false;
    const double n = sqrt((double)cam.W[0] * cam.W[0] + (double)cam.W[1] * cam.W[1] +
                          (double)cam.W[2] * cam.W[2]);
    int off = 0;  // components below 1e-3 of the direction's length
    for (int i = 0; i < 3; ++i) off += fabs((double)cam.W[i]) <= 1e-3 * n;
    return off == 2;
}

int render_segments(const svr_camera& cam, const VolDesc& v, const svr_params& p) {
    if (p.mode > SVR_MIPRGB || p.ratio != 0 || p.star_n != 0) return 1;
    if (axis_parallel(cam)) return 1;
    const double rays = (double)cam.width * cam.height;
    const double longest = sqrt((double)v.nx * v.nx + (double)v.ny * v.ny + (double)v.nz * v.nz) /
                           (double)p.dt;
    if (rays * longest < 16777216.0) return 1;
    const double want = ceil(2097152.0 / rays);
    const double most = floor(longest / 256.0);
    return (int)fmax(1.0, fmin(8.0, fmin(want, most)));
}

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

// Occupancy cap.  A launch given more than a third of the CU's 160 KiB of LDS runs at most
// two 256-lane workgroups (two waves per SIMD) per CU.  These kernels run faster so than at
// the three or four waves their registers allow, with images unchanged:
// - the plain AVIP_RGB march (1920x1080 views of the 512x512x1024 cube, dt 0.5: 2.80 -> 2.63
//   ms, and the L2 misses per frame 3.22 -> 2.92 GB; 16-bit storage and dt 1 11% faster);
// - the float32 split MIP marches with the out-of-range reuse loads (dt < 1): MIP0 2.34 ->
//   2.30 ms (3.18 -> 2.90 GB); MIP1 and MIP_RGB 2.57 ms with the reuse branch, with the reuse
//   loads at six fetch slots (128 VGPRs) 2.76 ms at four waves, 2.65 at three and 2.51 at
//   two, and 2.41 ms at eight slots (163 VGPRs) and two waves.
// At two waves, deeper pipelines (6 to 8 fetch slots for AVIP_RGB, 7 to 10 for MIP0) were
// slower again (2.74-2.76 / 2.39-2.47 ms), and at four waves (124 / 127 VGPRs) AVIP_RGB and
// MIP0 were 3-6% slower than at three: the gathers in flight per CU, not the waves to hide
// their latency, set the speed.  The other kernels are not capped: the box-smoothed
// marches, 16-bit MIP and AVIP0, the dt >= 1 views of uniform cubes and the line-ratio
// methods ran 5-29% slower with the cap.
constexpr size_t kTwoGroupsLds = 56 * 1024;

static size_t capped_lds(size_t need, bool cap) {
    return cap && need < kTwoGroupsLds ? kTwoGroupsLds : need;
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
    const int nseg = render_segments(cam, v->d, p);
    if (nseg > 1) {
        const int64_t npix = (int64_t)cam.width * cam.height;
        hipLaunchKernelGGL(split_clear_kernel, dim3((unsigned)((npix + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, stream, reinterpret_cast<unsigned long long*>(out),
                           npix);
        const bool box = p.box_arm > 0;
        SplitFn sf = pick_split_any(v->d.dtype, v->d.brick, wide, p.dt, p.mode, box);
        const size_t ring = box ? (size_t)(2 * p.box_arm + 1) * kBlock * sizeof(float) : 0;
        const bool cap = !box && v->d.dtype == SVR_F32 && p.dt < 1.0f && !wide;
        hipLaunchKernelGGL(sf, dim3((unsigned)(a.nblocks * nseg)), dim3(kBlock),
                           capped_lds(ring, cap), stream, a, nseg);
        const size_t lds = (size_t)(lut.n + 1) * sizeof(float4);
        RenderFn fin = p.mode == SVR_MIP0   ? split_finalize_kernel<SVR_MIP0>
                       : p.mode == SVR_MIP1 ? split_finalize_kernel<SVR_MIP1>
                                            : split_finalize_kernel<SVR_MIPRGB>;
        hipLaunchKernelGGL(fin, dim3(a.nblocks), dim3(kBlock), lds, stream, a);
        return hip_fail(hipGetLastError(), "render launch (split rays)");
    }
    RenderFn fn = pick_any(v->d.dtype, v->d.brick, wide, p.dt, smooth, p.mode, p.ratio);
    const bool cap = p.mode == SVR_AVIPRGB && smooth == kSmoothNone && p.ratio == 0;
    const size_t lds = capped_lds(render_lds_bytes(lut.n, p.box_arm, p.ratio), cap);
    hipLaunchKernelGGL(fn, dim3(a.nblocks), dim3(kBlock), lds, stream, a);
    return hip_fail(hipGetLastError(), "render launch");
}

}  // namespace svr
