// Separable 3D smoothing pre-pass (Section 4.2: the 1D kernel applied successively along
// each axis) and the voxel-wise line-ratio pass (Section 4.5).  Streaming, HBM-bound.
#include "common.h"

namespace svr {

struct Taps {
    float g[SVR_MAX_TAPS];
    int32_t n;
};

// Pass along x (contiguous): a workgroup stages one row segment plus its clamped halo in LDS.
template <int DT_IN>
__global__ __launch_bounds__(kBlock) void smooth_x_kernel(const typename Elem<DT_IN>::T* in,
                                                          float* out, int32_t nx, int32_t nseg,
                                                          const Taps taps) {
    __shared__ float tile[kBlock + SVR_MAX_TAPS];
    __shared__ float g[SVR_MAX_TAPS];
    const int T = taps.n, r = T / 2;
    const int64_t row = blockIdx.x / nseg;
    const int x0 = (blockIdx.x % nseg) * kBlock;
    const typename Elem<DT_IN>::T* src = in + row * nx;
    if (threadIdx.x < T) g[threadIdx.x] = taps.g[threadIdx.x];
    for (int i = threadIdx.x; i < kBlock + T - 1; i += kBlock) {
        int x = x0 - r + i;
        x = x < 0 ? 0 : (x > nx - 1 ? nx - 1 : x);
        tile[i] = Elem<DT_IN>::get(src, (uint32_t)x);
    }
    __syncthreads();
    const int x = x0 + threadIdx.x;
    if (x >= nx) return;
    float acc = 0.0f;
    for (int j = 0; j < T; ++j) acc = fmaf(g[j], tile[threadIdx.x + j], acc);
    out[row * nx + x] = acc;
}

// Pass along a strided axis: element (o, a, i) at o*n_axis*n_inner + a*n_inner + i.  Each lane
// produces R consecutive outputs along the axis from R + T - 1 inputs (register blocking);
// neighbouring lanes read neighbouring i, so every load is coalesced.
template <int DT_OUT, int R>
__global__ __launch_bounds__(kBlock) void smooth_axis_kernel(const float* in,
                                                             typename Elem<DT_OUT>::T* out,
                                                             int64_t n_inner, int32_t n_axis,
                                                             const Taps taps) {
    __shared__ float g[SVR_MAX_TAPS];
    const int T = taps.n, r = T / 2;
    if (threadIdx.x < T) g[threadIdx.x] = taps.g[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_inner) return;
    const int a0 = blockIdx.y * R;
    const int64_t base = (int64_t)blockIdx.z * n_axis * n_inner + i;
    float acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0f;
    for (int m = 0; m < R + T - 1; ++m) {
        int aa = a0 - r + m;
        aa = aa < 0 ? 0 : (aa > n_axis - 1 ? n_axis - 1 : aa);
        const float val = in[base + (int64_t)aa * n_inner];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int j = m - q;
            if (j >= 0 && j < T) acc[q] = fmaf(g[j], val, acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (a0 + q < n_axis) out[base + (int64_t)(a0 + q) * n_inner] = Elem<DT_OUT>::put(acc[q]);
}

constexpr int kAxisR = 8;

template <int DT_OUT>
static void axis_launch(const float* in, void* out, int64_t n_inner, int n_axis, int n_outer,
                        const Taps& t, hipStream_t stream) {
    const dim3 grid((unsigned)((n_inner + kBlock - 1) / kBlock),
                    (unsigned)((n_axis + kAxisR - 1) / kAxisR), (unsigned)n_outer);
    hipLaunchKernelGGL((smooth_axis_kernel<DT_OUT, kAxisR>), grid, dim3(kBlock), 0, stream, in,
                       (typename Elem<DT_OUT>::T*)out, n_inner, n_axis, t);
}

svr_status launch_smooth(const svr_cube_view& c, const float* taps_host, int ntaps, void* out,
                         void* ws, hipStream_t stream) {
    Taps t;
    for (int j = 0; j < ntaps; ++j) t.g[j] = taps_host[j];
    t.n = ntaps;
    const int64_t nvox = (int64_t)c.nx * c.ny * c.nz;
    float* w0 = static_cast<float*>(ws);
    float* w1 = w0 + nvox;
    const int nseg = (c.nx + kBlock - 1) / kBlock;
    const dim3 gx((unsigned)((int64_t)nseg * c.ny * c.nz));
    switch (c.dtype) {
        case SVR_F16:
            hipLaunchKernelGGL(smooth_x_kernel<SVR_F16>, gx, dim3(kBlock), 0, stream,
                               (const _Float16*)c.data, w0, c.nx, nseg, t);
            break;
        case SVR_BF16:
            hipLaunchKernelGGL(smooth_x_kernel<SVR_BF16>, gx, dim3(kBlock), 0, stream,
                               (const uint16_t*)c.data, w0, c.nx, nseg, t);
            break;
        default:
            hipLaunchKernelGGL(smooth_x_kernel<SVR_F32>, gx, dim3(kBlock), 0, stream,
                               (const float*)c.data, w0, c.nx, nseg, t);
    }
    axis_launch<SVR_F32>(w0, w1, c.nx, c.ny, c.nz, t, stream);  // along y
    const int64_t plane = (int64_t)c.nx * c.ny;
    switch (c.dtype) {  // along z, converting to the output type
        case SVR_F16: axis_launch<SVR_F16>(w1, out, plane, c.nz, 1, t, stream); break;
        case SVR_BF16: axis_launch<SVR_BF16>(w1, out, plane, c.nz, 1, t, stream); break;
        default: axis_launch<SVR_F32>(w1, out, plane, c.nz, 1, t, stream);
    }
    return hip_fail(hipGetLastError(), "smooth launch");
}

// ------------------------------------------------------------------------- line ratio
template <int DT>
__global__ __launch_bounds__(kBlock) void line_ratio_kernel(const typename Elem<DT>::T* cube,
                                                            int32_t nx, int64_t sx, int64_t sy,
                                                            int64_t sz, int32_t z0a, int32_t z0b,
                                                            float min_a, float min_b,
                                                            float datamin, float* out,
                                                            int32_t ny) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, j = blockIdx.z;
    const int64_t off = (int64_t)y * sy + (int64_t)x * sx;
    float a = Elem<DT>::get(cube + (int64_t)(z0a + j) * sz + off, 0);
    float b = Elem<DT>::get(cube + (int64_t)(z0b + j) * sz + off, 0);
    if (a < min_a) a = datamin;
    if (b < min_b) b = datamin;
    out[((int64_t)j * ny + y) * nx + x] = a > 0.0f ? b / a : datamin;
}

svr_status launch_line_ratio(const svr_cube_view& c, int z0a, int z0b, int nzw, float min_a,
                             float min_b, float datamin, float* out, hipStream_t stream) {
    const bool contig = c.sx == 0 && c.sy == 0 && c.sz == 0;
    const int64_t sx = contig ? 1 : c.sx;
    const int64_t sy = contig ? (int64_t)c.nx : c.sy;
    const int64_t sz = contig ? (int64_t)c.nx * c.ny : c.sz;
    const dim3 grid((unsigned)((c.nx + kBlock - 1) / kBlock), (unsigned)c.ny, (unsigned)nzw);
    switch (c.dtype) {
        case SVR_F16:
            hipLaunchKernelGGL(line_ratio_kernel<SVR_F16>, grid, dim3(kBlock), 0, stream,
                               (const _Float16*)c.data, c.nx, sx, sy, sz, z0a, z0b, min_a, min_b,
                               datamin, out, c.ny);
            break;
        case SVR_BF16:
            hipLaunchKernelGGL(line_ratio_kernel<SVR_BF16>, grid, dim3(kBlock), 0, stream,
                               (const uint16_t*)c.data, c.nx, sx, sy, sz, z0a, z0b, min_a, min_b,
                               datamin, out, c.ny);
            break;
        default:
            hipLaunchKernelGGL(line_ratio_kernel<SVR_F32>, grid, dim3(kBlock), 0, stream,
                               (const float*)c.data, c.nx, sx, sy, sz, z0a, z0b, min_a, min_b,
                               datamin, out, c.ny);
    }
    return hip_fail(hipGetLastError(), "line_ratio launch");
}

}  // namespace svr
