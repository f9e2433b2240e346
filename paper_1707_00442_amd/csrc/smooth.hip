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

// Any odd tap count: x pass through an LDS row, then y and z with register blocking.
static svr_status launch_smooth_generic(const svr_cube_view& c, const float* taps_host,
                                        int ntaps, void* out, void* ws, hipStream_t stream) {
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

// ---------------------------------------------------------------- fixed tap counts
// For the common tap counts (the 5-, 9- and 13-tap binomials, the sigma = 1, 2, 3 Gaussians
// of 7, 13 and 19 taps) the passes are two streaming kernels with compile-time loops:
//   * x and y fused: a workgroup stages one z-slice tile of the input with its clamped halo
//     in LDS, filters it along x into a second LDS tile, then along y to float32 output;
//   * z: every lane produces 16 consecutive outputs of one (y, x) column from 15 + T
//     inputs read straight from memory (neighbouring lanes read neighbouring x).
// Each output is the same ordered sum sum_j g[j] v[j] (fma from j = 0 up) as in the generic
// kernels; only products inside the kernel's support are formed.  Taps are kernel
// arguments indexed with compile-time offsets, so they sit in scalar registers.
template <int T>
struct FixedTaps {
    float g[T];
};

// acc[q] = sum_{j<T} g[j] v[q + j] for q < R, from the stream v[0 .. R+T-2] delivered by
// fetch(m), each product formed once and accumulated in increasing j.
template <int T, int R, class Fetch>
__device__ __forceinline__ void conv_block(const FixedTaps<T>& g, Fetch&& fetch, float (&acc)[R]) {
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0f;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        // acc[q] += g[j] * v[q + j]: the input index runs over j .. j+R-1
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] = fmaf(g.g[j], fetch(q + j), acc[q]);
    }
}

constexpr int kXyTx = 64;  // tile width (x)
constexpr int kXyTy = 32;  // tile height (y)
constexpr int kXyR = 8;    // outputs per lane along x (first phase) and along y (second)

template <int T>
constexpr int xy_lds_floats() {
    return (kXyTy + T - 1) * (kXyTx + T - 1) + (kXyTy + T - 1) * kXyTx;
}

template <int DT_IN, int T>
__global__ __launch_bounds__(kBlock) void smooth_xy_kernel(const typename Elem<DT_IN>::T* in,
                                                           float* out, int32_t nx, int32_t ny,
                                                           int32_t tiles_x, int32_t tiles_y,
                                                           const FixedTaps<T> g) {
    constexpr int r = T / 2;
    constexpr int AW = kXyTx + T - 1, AH = kXyTy + T - 1;
    __shared__ float A[AH * AW];
    __shared__ float B[AH * kXyTx];
    const int64_t t = blockIdx.x;
    const int tx = (int)(t % tiles_x);
    const int ty = (int)((t / tiles_x) % tiles_y);
    const int64_t z = t / ((int64_t)tiles_x * tiles_y);
    const int x0 = tx * kXyTx, y0 = ty * kXyTy;
    const typename Elem<DT_IN>::T* slice = in + z * ny * nx;
    // input tile with clamp-to-edge halo
    for (int i = threadIdx.x; i < AH * AW; i += kBlock) {
        const int ry = i / AW, rx = i - ry * AW;
        int gx = x0 - r + rx, gy = y0 - r + ry;
        gx = gx < 0 ? 0 : (gx > nx - 1 ? nx - 1 : gx);
        gy = gy < 0 ? 0 : (gy > ny - 1 ? ny - 1 : gy);
        A[i] = Elem<DT_IN>::get(slice, (uint32_t)(gy * nx + gx));
    }
    __syncthreads();
    // along x: rows 0 .. AH-1, eight lanes per row, kXyR outputs each
    {
        const int xg = (threadIdx.x & 7) * kXyR;
        for (int ry = threadIdx.x >> 3; ry < AH; ry += kBlock / 8) {
            const float* a = A + ry * AW + xg;
            float acc[kXyR];
            conv_block<T, kXyR>(g, [&](int m) { return a[m]; }, acc);
#pragma unroll
            for (int q = 0; q < kXyR; ++q) B[ry * kXyTx + xg + q] = acc[q];
        }
    }
    __syncthreads();
    // along y: 64 columns x 4 groups of kXyR rows
    {
        const int x = threadIdx.x & (kXyTx - 1);
        const int yg = (threadIdx.x >> 6) * kXyR;
        const float* b = B + yg * kXyTx + x;
        float acc[kXyR];
        conv_block<T, kXyR>(g, [&](int m) { return b[m * kXyTx]; }, acc);
        const int gx = x0 + x;
        if (gx < nx) {
#pragma unroll
            for (int q = 0; q < kXyR; ++q) {
                const int gy = y0 + yg + q;
                if (gy < ny) out[(z * ny + gy) * nx + gx] = acc[q];
            }
        }
    }
}

constexpr int kZR = 16;  // outputs per lane along z

// Along z (stride plane = nx*ny): lane i of block (column block cb, z block zb) filters column
// cb*256 + i for outputs zb*kZR .. zb*kZR+kZR-1.  Blocks are numbered with the z block fastest
// and dealt to XCDs in contiguous runs, so the T-1 halo planes shared by neighbouring z blocks
// are re-read from the same L2.
template <int DT_OUT, int T>
__global__ __launch_bounds__(kBlock) void smooth_z_kernel(const float* in,
                                                          typename Elem<DT_OUT>::T* out,
                                                          int64_t plane, int32_t nz,
                                                          int32_t zblocks, int32_t nblocks,
                                                          const FixedTaps<T> g) {
    constexpr int r = T / 2;
    const int b = xcd_tile((int)blockIdx.x, nblocks);
    const int zb = b % zblocks;
    const int64_t i = (int64_t)(b / zblocks) * kBlock + threadIdx.x;
    if (i >= plane) return;
    const int z0 = zb * kZR;
    const float* col = in + i;
    float acc[kZR];
    conv_block<T, kZR>(g, [&](int m) {
        int zz = z0 - r + m;
        zz = zz < 0 ? 0 : (zz > nz - 1 ? nz - 1 : zz);
        return col[(int64_t)zz * plane];
    }, acc);
#pragma unroll
    for (int q = 0; q < kZR; ++q)
        if (z0 + q < nz) out[(int64_t)(z0 + q) * plane + i] = Elem<DT_OUT>::put(acc[q]);
}

template <int T>
static svr_status smooth_fixed(const svr_cube_view& c, const float* taps_host, void* out,
                               float* w0, hipStream_t stream) {
    FixedTaps<T> g;
    for (int j = 0; j < T; ++j) g.g[j] = taps_host[j];
    const int tiles_x = (c.nx + kXyTx - 1) / kXyTx, tiles_y = (c.ny + kXyTy - 1) / kXyTy;
    const dim3 gxy((unsigned)((int64_t)tiles_x * tiles_y * c.nz));
    switch (c.dtype) {
        case SVR_F16:
            hipLaunchKernelGGL((smooth_xy_kernel<SVR_F16, T>), gxy, dim3(kBlock), 0, stream,
                               (const _Float16*)c.data, w0, c.nx, c.ny, tiles_x, tiles_y, g);
            break;
        case SVR_BF16:
            hipLaunchKernelGGL((smooth_xy_kernel<SVR_BF16, T>), gxy, dim3(kBlock), 0, stream,
                               (const uint16_t*)c.data, w0, c.nx, c.ny, tiles_x, tiles_y, g);
            break;
        default:
            hipLaunchKernelGGL((smooth_xy_kernel<SVR_F32, T>), gxy, dim3(kBlock), 0, stream,
                               (const float*)c.data, w0, c.nx, c.ny, tiles_x, tiles_y, g);
    }
    const int64_t plane = (int64_t)c.nx * c.ny;
    const int zblocks = (c.nz + kZR - 1) / kZR;
    const int64_t nb = (plane + kBlock - 1) / kBlock * zblocks;
    if (nb > 0x7fffffff) return SVR_EUNSUPPORTED;
    const dim3 gz((unsigned)nb);
    switch (c.dtype) {
        case SVR_F16:
            hipLaunchKernelGGL((smooth_z_kernel<SVR_F16, T>), gz, dim3(kBlock), 0, stream, w0,
                               (_Float16*)out, plane, c.nz, zblocks, (int)nb, g);
            break;
        case SVR_BF16:
            hipLaunchKernelGGL((smooth_z_kernel<SVR_BF16, T>), gz, dim3(kBlock), 0, stream, w0,
                               (uint16_t*)out, plane, c.nz, zblocks, (int)nb, g);
            break;
        default:
            hipLaunchKernelGGL((smooth_z_kernel<SVR_F32, T>), gz, dim3(kBlock), 0, stream, w0,
                               (float*)out, plane, c.nz, zblocks, (int)nb, g);
    }
    return hip_fail(hipGetLastError(), "smooth launch");
}

svr_status launch_smooth(const svr_cube_view& c, const float* taps_host, int ntaps, void* out,
                         void* ws, hipStream_t stream) {
    float* w0 = static_cast<float*>(ws);
    switch (ntaps) {
        case 5: return smooth_fixed<5>(c, taps_host, out, w0, stream);
        case 7: return smooth_fixed<7>(c, taps_host, out, w0, stream);
        case 9: return smooth_fixed<9>(c, taps_host, out, w0, stream);
        case 13: return smooth_fixed<13>(c, taps_host, out, w0, stream);
        case 19: return smooth_fixed<19>(c, taps_host, out, w0, stream);
        default: break;
    }
    return launch_smooth_generic(c, taps_host, ntaps, out, ws, stream);
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
