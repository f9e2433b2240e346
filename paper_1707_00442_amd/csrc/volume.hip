// Upload path: finite min/max reduction, brick + apron + quantise, and export back to a
// linear cube.  All three stream the cube once and are HBM-bound.
#include <math.h>

#include "common.h"

namespace svr {

constexpr int kMinmaxMaxBlocks = 2048;

// Per-workgroup partial (min, max, any non-finite) over a strided cube viewed as rows of
// nx elements: row = z * ny + y (a C-contiguous cube is passed as one long row).
template <int DT>
__global__ __launch_bounds__(kBlock) void minmax_partial(const typename Elem<DT>::T* src,
                                                         int64_t nx, int64_t nrows, int64_t ny,
                                                         int64_t sx, int64_t sy, int64_t sz,
                                                         float* partial) {
    float lo = INFINITY, hi = -INFINITY, bad = 0.0f;
    const int64_t xs = (int64_t)gridDim.x * kBlock;
    for (int64_t row = blockIdx.y; row < nrows; row += gridDim.y) {
        const int64_t base = (row / ny) * sz + (row % ny) * sy;
        for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < nx; x += xs) {
            const float v = Elem<DT>::get(src + base + x * sx, 0);
            if (isfinite(v)) {
                lo = fminf(lo, v);
                hi = fmaxf(hi, v);
            } else {
                bad = 1.0f;
            }
        }
    }
    // wave reduction then across the 4 waves
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o));
        hi = fmaxf(hi, __shfl_xor(hi, o));
        bad = fmaxf(bad, __shfl_xor(bad, o));
    }
    __shared__ float s[3][kBlock / kWave];
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s[0][w] = lo;
        s[1][w] = hi;
        s[2][w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / kWave; ++i) {
            lo = fminf(lo, s[0][i]);
            hi = fmaxf(hi, s[1][i]);
            bad = fmaxf(bad, s[2][i]);
        }
        const int b = blockIdx.y * gridDim.x + blockIdx.x;
        partial[3 * b + 0] = lo;
        partial[3 * b + 1] = hi;
        partial[3 * b + 2] = bad;
    }
}

// Reduce the partials.  raw != 0: out = (finite min, finite max) or NaN pair.  raw == 0
// (volume): out = (min, max) of the values as stored -- non-finite voxels replaced by the
// fill value (nan_fill, or the finite minimum when nan_fill is NaN, or 0 when no value is
// finite) -- each rounded to the storage type; out[2] = the fill value.
template <int DT_OUT>
__global__ __launch_bounds__(kBlock) void minmax_final(const float* partial, int nparts,
                                                       int raw, float nan_fill, float* out) {
    float lo = INFINITY, hi = -INFINITY, bad = 0.0f;
    for (int i = threadIdx.x; i < nparts; i += kBlock) {
        lo = fminf(lo, partial[3 * i]);
        hi = fmaxf(hi, partial[3 * i + 1]);
        bad = fmaxf(bad, partial[3 * i + 2]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o));
        hi = fmaxf(hi, __shfl_xor(hi, o));
        bad = fmaxf(bad, __shfl_xor(bad, o));
    }
    __shared__ float s[3][kBlock / kWave];
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        s[0][w] = lo;
        s[1][w] = hi;
        s[2][w] = bad;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < kBlock / kWave; ++i) {
        lo = fminf(lo, s[0][i]);
        hi = fmaxf(hi, s[1][i]);
        bad = fmaxf(bad, s[2][i]);
    }
    const bool any = lo <= hi;
    if (raw) {
        out[0] = any ? lo : NAN;
        out[1] = any ? hi : NAN;
        return;
    }
    float fill = isnan(nan_fill) ? (any ? lo : 0.0f) : nan_fill;
    if (bad > 0.0f) {
        lo = any ? fminf(lo, fill) : fill;
        hi = any ? fmaxf(hi, fill) : fill;
    }
    using T = typename Elem<DT_OUT>::T;
    const T ql = Elem<DT_OUT>::put(lo), qh = Elem<DT_OUT>::put(hi), qf = Elem<DT_OUT>::put(fill);
    out[0] = Elem<DT_OUT>::get(&ql, 0);
    out[1] = Elem<DT_OUT>::get(&qh, 0);
    out[2] = Elem<DT_OUT>::get(&qf, 0);
}

// One workgroup per brick: gather its E^3 voxels (clamped to the cube), replace non-finite
// values by the fill value, convert to the storage type, write the brick contiguously.
template <int DT_IN, int DT_OUT, int C>
__global__ __launch_bounds__(kBlock) void brick_kernel(const typename Elem<DT_IN>::T* src,
                                                       int64_t sx, int64_t sy, int64_t sz,
                                                       VolDesc dst, const float* aux) {
    constexpr int E = C + 1;
    constexpr int E3 = E * E * E;
    using TO = typename Elem<DT_OUT>::T;
    const uint32_t b = blockIdx.x;
    const uint32_t bx = b % (uint32_t)dst.nbx;
    const uint32_t by = (b / (uint32_t)dst.nbx) % (uint32_t)dst.nby;
    const uint32_t bz = b / ((uint32_t)dst.nbx * (uint32_t)dst.nby);
    const float fill = aux[2];
    TO* out = (TO*)dst.data + (size_t)b * dst.pitch;
    for (uint32_t e = threadIdx.x; e < dst.pitch; e += kBlock) {
        if (e >= (uint32_t)E3) {
            out[e] = Elem<DT_OUT>::put(0.0f);
            continue;
        }
        const uint32_t lx = e % E, ly = (e / E) % E, lz = e / (E * E);
        const int64_t gx = min((int64_t)(bx * C + lx), (int64_t)dst.nx - 1);
        const int64_t gy = min((int64_t)(by * C + ly), (int64_t)dst.ny - 1);
        const int64_t gz = min((int64_t)(bz * C + lz), (int64_t)dst.nz - 1);
        float v = Elem<DT_IN>::get(src + gz * sz + gy * sy + gx * sx, 0);
        if (!isfinite(v)) v = fill;
        out[e] = Elem<DT_OUT>::put(v);
    }
}

// Bricked storage -> C-contiguous [z][y][x] of the storage type.
template <int DT, int C>
__global__ __launch_bounds__(kBlock) void export_kernel(VolDesc v, typename Elem<DT>::T* out) {
    constexpr int E = C + 1;
    constexpr int SH = C == 8 ? 3 : 4;
    using T = typename Elem<DT>::T;
    const uint32_t x = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    if (x >= (uint32_t)v.nx) return;
    const uint32_t b = ((z >> SH) * (uint32_t)v.nby + (y >> SH)) * (uint32_t)v.nbx + (x >> SH);
    const uint32_t loc = ((z & (C - 1)) * E + (y & (C - 1))) * E + (x & (C - 1));
    out[((size_t)z * v.ny + y) * v.nx + x] = ((const T*)v.data)[(size_t)b * v.pitch + loc];
}

static void minmax_grid(const svr_cube_view& c, int64_t& nx, int64_t& nrows, int64_t& ny,
                        int64_t& sx, int64_t& sy, int64_t& sz, dim3& grid) {
    const bool contig = c.sx == 0 && c.sy == 0 && c.sz == 0;
    if (contig) {
        nx = (int64_t)c.nx * c.ny * c.nz;
        nrows = 1;
        ny = 1;
        sx = 1;
        sy = 0;
        sz = 0;
    } else {
        nx = c.nx;
        nrows = (int64_t)c.ny * c.nz;
        ny = c.ny;
        sx = c.sx;
        sy = c.sy;
        sz = c.sz;
    }
    int64_t gx = (nx + kBlock * 8 - 1) / (kBlock * 8);
    gx = gx < 1 ? 1 : (gx > kMinmaxMaxBlocks ? kMinmaxMaxBlocks : gx);
    int64_t gy = kMinmaxMaxBlocks / gx;
    gy = gy < 1 ? 1 : (gy > nrows ? nrows : gy);
    grid = dim3((unsigned)gx, (unsigned)gy);
}

size_t minmax_partial_floats() { return 3 * (size_t)kMinmaxMaxBlocks; }

svr_status launch_minmax(const svr_cube_view& c, float* partial, float* out, int raw,
                         int out_dtype, float nan_fill, hipStream_t stream) {
    int64_t nx, nrows, ny, sx, sy, sz;
    dim3 grid;
    minmax_grid(c, nx, nrows, ny, sx, sy, sz, grid);
    switch (c.dtype) {
        case SVR_F16:
            hipLaunchKernelGGL(minmax_partial<SVR_F16>, grid, dim3(kBlock), 0, stream,
                               (const _Float16*)c.data, nx, nrows, ny, sx, sy, sz, partial);
            break;
        case SVR_BF16:
            hipLaunchKernelGGL(minmax_partial<SVR_BF16>, grid, dim3(kBlock), 0, stream,
                               (const uint16_t*)c.data, nx, nrows, ny, sx, sy, sz, partial);
            break;
        default:
            hipLaunchKernelGGL(minmax_partial<SVR_F32>, grid, dim3(kBlock), 0, stream,
                               (const float*)c.data, nx, nrows, ny, sx, sy, sz, partial);
    }
    const int nparts = (int)(grid.x * grid.y);
    switch (out_dtype) {
        case SVR_F16:
            hipLaunchKernelGGL(minmax_final<SVR_F16>, dim3(1), dim3(kBlock), 0, stream, partial,
                               nparts, raw, nan_fill, out);
            break;
        case SVR_BF16:
            hipLaunchKernelGGL(minmax_final<SVR_BF16>, dim3(1), dim3(kBlock), 0, stream, partial,
                               nparts, raw, nan_fill, out);
            break;
        default:
            hipLaunchKernelGGL(minmax_final<SVR_F32>, dim3(1), dim3(kBlock), 0, stream, partial,
                               nparts, raw, nan_fill, out);
    }
    return hip_fail(hipGetLastError(), "minmax launch");
}

template <int DT_IN, int DT_OUT>
static void brick_launch(const svr_cube_view& c, const VolDesc& d, const float* aux,
                         hipStream_t stream) {
    const int64_t sx = c.sx == 0 && c.sy == 0 && c.sz == 0 ? 1 : c.sx;
    const int64_t sy = c.sx == 0 && c.sy == 0 && c.sz == 0 ? (int64_t)c.nx : c.sy;
    const int64_t sz = c.sx == 0 && c.sy == 0 && c.sz == 0 ? (int64_t)c.nx * c.ny : c.sz;
    const dim3 grid((unsigned)((int64_t)d.nbx * d.nby * d.nbz));
    using TI = typename Elem<DT_IN>::T;
    if (d.brick == 16)
        hipLaunchKernelGGL((brick_kernel<DT_IN, DT_OUT, 16>), grid, dim3(kBlock), 0, stream,
                           (const TI*)c.data, sx, sy, sz, d, aux);
    else
        hipLaunchKernelGGL((brick_kernel<DT_IN, DT_OUT, 8>), grid, dim3(kBlock), 0, stream,
                           (const TI*)c.data, sx, sy, sz, d, aux);
}

template <int DT_IN>
static void brick_launch_in(const svr_cube_view& c, const VolDesc& d, const float* aux,
                            hipStream_t stream) {
    if (d.dtype == SVR_F16) brick_launch<DT_IN, SVR_F16>(c, d, aux, stream);
    else if (d.dtype == SVR_BF16) brick_launch<DT_IN, SVR_BF16>(c, d, aux, stream);
    else brick_launch<DT_IN, SVR_F32>(c, d, aux, stream);
}

svr_status launch_brick(const svr_cube_view& c, const VolDesc& d, const float* aux,
                        hipStream_t stream) {
    if (c.dtype == SVR_F16) brick_launch_in<SVR_F16>(c, d, aux, stream);
    else if (c.dtype == SVR_BF16) brick_launch_in<SVR_BF16>(c, d, aux, stream);
    else brick_launch_in<SVR_F32>(c, d, aux, stream);
    return hip_fail(hipGetLastError(), "brick launch");
}

svr_status launch_export(const VolDesc& d, void* out, hipStream_t stream) {
    const dim3 grid((unsigned)((d.nx + kBlock - 1) / kBlock), (unsigned)d.ny, (unsigned)d.nz);
#define SVR_EXPORT(DT, C)                                                                   \
    hipLaunchKernelGGL((export_kernel<DT, C>), grid, dim3(kBlock), 0, stream, d,             \
                       (typename Elem<DT>::T*)out)
    if (d.brick == 16) {
        if (d.dtype == SVR_F16) SVR_EXPORT(SVR_F16, 16);
        else if (d.dtype == SVR_BF16) SVR_EXPORT(SVR_BF16, 16);
        else SVR_EXPORT(SVR_F32, 16);
    } else {
        if (d.dtype == SVR_F16) SVR_EXPORT(SVR_F16, 8);
        else if (d.dtype == SVR_BF16) SVR_EXPORT(SVR_BF16, 8);
        else SVR_EXPORT(SVR_F32, 8);
    }
#undef SVR_EXPORT
    return hip_fail(hipGetLastError(), "export launch");
}

}  // namespace svr
