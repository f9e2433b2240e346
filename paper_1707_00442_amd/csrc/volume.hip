// Upload path: finite min/max of a cube view, the one-pass upload (brick + apron + quantise
// + min/max), and export back to a linear cube.  All stream the cube once; HBM-bound.
#include <math.h>

#include <mutex>

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

// ------------------------------------------------------------------ one-pass upload
// The upload reads the cube once:
//   upload_init       clears the reduction slots (one lane);
//   brick_group       one workgroup per run of G bricks along x stages the 9 x 9 x (G C + 1)
//                     source slab (clamped to the cube) in LDS, writes the G bricks as one
//                     contiguous run (apron and pitch padding included), and folds the
//                     slab's finite min/max and a non-finite flag into one of 256 slot
//                     triples with integer atomics on an order-preserving encoding;
//                     non-finite voxels are stored as NaN;
//   upload_final      folds the slots into (min, max, fill) of the stored values, as
//                     minmax_final does for a separate reduction, plus the flag;
//   upload_fill       replaces the stored NaNs by the fill value; every workgroup returns at
//                     once when the cube had no non-finite voxel.
// aux: [0] min, [1] max, [2] fill (storage-rounded), [3] non-finite flag, [4..) slots.

// float -> uint32 with the same order for every non-NaN value
__device__ __forceinline__ uint32_t order_enc(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float order_dec(uint32_t e) {
    return __uint_as_float((e & 0x80000000u) ? (e & 0x7fffffffu) : ~e);
}

// The reduction slots: kSlots copies of (min, max, non-finite) so that the workgroups'
// atomics spread over many addresses (same-address atomics serialise in one L2 channel).
constexpr int kSlots = 256;

__global__ void upload_init(uint32_t* slots) {
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
        slots[i] = 0xffffffffu;           // min (encoded)
        slots[kSlots + i] = 0u;           // max (encoded)
        slots[2 * kSlots + i] = 0u;       // non-finite seen
    }
}

template <int C>
struct BrickGroup {
    static constexpr int E = C + 1;
    static constexpr int G = C == 8 ? 8 : 2;   // bricks per workgroup along x
    static constexpr int W = G * C + 1;        // staged slab width (x)
    static constexpr int WP = (W + 3) / 4 * 4; // LDS row pitch (16-byte rows)
    static constexpr int TILE = E * E * WP;    // 22 KB (C = 8) or 41 KB (C = 16) of floats
};

// 16-byte vector of a storage type
template <class T>
struct alignas(16) Vec16 {
    static constexpr int N = 16 / sizeof(T);
    T v[N];
};

template <int DT_IN, int DT_OUT, int C, bool CONTIG>
__global__ __launch_bounds__(kBlock) void brick_group_kernel(const typename Elem<DT_IN>::T* src,
                                                             int64_t sx, int64_t sy, int64_t sz,
                                                             VolDesc dst, int32_t groups_x,
                                                             int32_t nblocks, int32_t vec_in,
                                                             uint32_t* slots) {
    using BG = BrickGroup<C>;
    constexpr int E = BG::E, G = BG::G, W = BG::W, WP = BG::WP, TILE = BG::TILE;
    constexpr int NW = kBlock / kWave;
    using TI = typename Elem<DT_IN>::T;
    using TO = typename Elem<DT_OUT>::T;
    constexpr int VI = Vec16<TI>::N, VO = Vec16<TO>::N;
    __shared__ __align__(16) float tile[TILE];
    __shared__ uint32_t s_red[3][NW];
    __shared__ int64_t s_row[E * E];
    const int t = xcd_tile((int)blockIdx.x, nblocks);
    const int gx = t % groups_x;
    const int rest = t / groups_x;
    const int by = rest % dst.nby, bz = rest / dst.nby;
    const int bx0 = gx * G;
    const int x0 = bx0 * C, y0 = by * C, z0 = bz * C;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    // element offsets of the E x E source rows (clamped to the cube)
    for (int row = threadIdx.x; row < E * E; row += kBlock) {
        const int lz = row / E, ly = row - lz * E;
        const int64_t gy = min(y0 + ly, dst.ny - 1), gz = min(z0 + lz, dst.nz - 1);
        s_row[row] = gz * sz + gy * sy;
    }
    __syncthreads();
    float lo = INFINITY, hi = -INFINITY;
    uint32_t bad = 0;
    auto take = [&](float v) -> float {
        if (isfinite(v)) {
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
            return v;
        }
        bad = 1;
        return NAN;
    };
    // vector path: contiguous rows, the group's G*C voxels inside the cube and aligned
    const bool vec = CONTIG && vec_in && x0 + G * C <= dst.nx;
    if (vec) {
        constexpr int PER_ROW = G * C / VI;          // vectors per row (the apron column apart)
        constexpr int NV = E * E * PER_ROW;
        constexpr int NLD = (NV + kBlock - 1) / kBlock;
        Vec16<TI> buf[NLD];
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + j * kBlock;
            if (i < NV) {
                const int row = i / PER_ROW, q = i - row * PER_ROW;
                buf[j] = *reinterpret_cast<const Vec16<TI>*>(src + s_row[row] + x0 + q * VI);
            }
        }
        // the apron column x0 + G C (clamped), one element per row: E * E rows (289 for
        // 16-voxel bricks, more than the workgroup's lanes)
        constexpr int NAP = (E * E + kBlock - 1) / kBlock;
        float ap[NAP];
#pragma unroll
        for (int j = 0; j < NAP; ++j) {
            const int row = threadIdx.x + j * kBlock;
            ap[j] = row < E * E ? Elem<DT_IN>::get(src + s_row[row],
                                                   (uint32_t)min(x0 + G * C, dst.nx - 1))
                                : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + j * kBlock;
            if (i < NV) {
                const int row = i / PER_ROW, q = i - row * PER_ROW;
                float f[VI];
#pragma unroll
                for (int m = 0; m < VI; ++m) f[m] = take(Elem<DT_IN>::get(buf[j].v, m));
                float* dstp = tile + row * WP + q * VI;
#pragma unroll
                for (int m = 0; m < VI; m += 4)
                    *reinterpret_cast<float4*>(dstp + m) = make_float4(f[m], f[m + 1], f[m + 2], f[m + 3]);
            }
        }
#pragma unroll
        for (int j = 0; j < NAP; ++j) {
            const int row = threadIdx.x + j * kBlock;
            if (row < E * E) tile[row * WP + G * C] = take(ap[j]);
        }
    } else {
        constexpr int NLD = (E * E * W + kBlock - 1) / kBlock;
        float vals[NLD];
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + j * kBlock;
            vals[j] = 0.0f;
            if (i < E * E * W) {
                const int row = i / W, lx = i - row * W;
                const int64_t gxx = min(x0 + lx, dst.nx - 1);
                vals[j] = Elem<DT_IN>::get(src + s_row[row] + (CONTIG ? gxx : gxx * sx), 0);
            }
        }
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + j * kBlock;
            if (i < E * E * W) {
                const int row = i / W, lx = i - row * W;
                tile[row * WP + lx] = take(vals[j]);
            }
        }
    }
    __syncthreads();
    // the run of bricks, 16 bytes per store: element l of brick k comes from
    // tile[(lz E + ly) WP + k C + lx] (0 in the pitch padding)
    const int nb = min(G, dst.nbx - bx0);
    TO* out = (TO*)dst.data + ((size_t)((size_t)bz * dst.nby + by) * dst.nbx + bx0) * dst.pitch;
    const uint32_t pvec = dst.pitch / VO;  // vectors per brick (the pitch is a multiple of 64)
    for (uint32_t q = threadIdx.x; q < pvec; q += kBlock) {
        int off[VO];
#pragma unroll
        for (int m = 0; m < VO; ++m) {
            const int l = (int)q * VO + m;
            if constexpr (DT_OUT == SVR_F32) {
                const int lz = l / (E * E), ly = (l / E) % E, lx = l % E;
                off[m] = l < E * E * E ? (lz * E + ly) * WP + lx : -1;
            } else {  // y-pairs: element 2 p + h of pair p = (lz C + ly) E + lx is voxel ly + h
                const int p = l >> 1, h = l & 1;
                const int lz = p / (C * E), ly = (p / E) % C, lx = p % E;
                off[m] = p < E * C * E ? (lz * E + ly + h) * WP + lx : -1;
            }
        }
        for (int k = 0; k < nb; ++k) {
            Vec16<TO> o;
#pragma unroll
            for (int m = 0; m < VO; ++m) o.v[m] = Elem<DT_OUT>::put(off[m] >= 0 ? tile[off[m] + k * C] : 0.0f);
            *reinterpret_cast<Vec16<TO>*>(out + (size_t)k * dst.pitch + (size_t)q * VO) = o;
        }
    }
    // workgroup reduction, then one atomic per slot
    uint32_t elo = lo <= hi ? order_enc(lo) : 0xffffffffu;
    uint32_t ehi = lo <= hi ? order_enc(hi) : 0u;
    for (int o = 32; o > 0; o >>= 1) {
        elo = min(elo, (uint32_t)__shfl_xor((int)elo, o));
        ehi = max(ehi, (uint32_t)__shfl_xor((int)ehi, o));
        bad |= (uint32_t)__shfl_xor((int)bad, o);
    }
    if (lane == 0) {
        s_red[0][wave] = elo;
        s_red[1][wave] = ehi;
        s_red[2][wave] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NW; ++i) {
            elo = min(elo, s_red[0][i]);
            ehi = max(ehi, s_red[1][i]);
            bad |= s_red[2][i];
        }
        const int sl = blockIdx.x & (kSlots - 1);
        atomicMin(&slots[sl], elo);
        atomicMax(&slots[kSlots + sl], ehi);
        if (bad) atomicOr(&slots[2 * kSlots + sl], 1u);
    }
}

template <int DT_OUT>
__global__ void upload_final(float* aux, float nan_fill) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t* slots = reinterpret_cast<const uint32_t*>(aux + 4);
    uint32_t elo = 0xffffffffu, ehi = 0u, nonfinite = 0u;
    for (int i = 0; i < kSlots; ++i) {
        elo = min(elo, slots[i]);
        ehi = max(ehi, slots[kSlots + i]);
        nonfinite |= slots[2 * kSlots + i];
    }
    const bool any = elo <= ehi;
    float lo = any ? order_dec(elo) : INFINITY;
    float hi = any ? order_dec(ehi) : -INFINITY;
    const bool bad = nonfinite != 0;
    const float fill = isnan(nan_fill) ? (any ? lo : 0.0f) : nan_fill;
    if (bad) {
        lo = any ? fminf(lo, fill) : fill;
        hi = any ? fmaxf(hi, fill) : fill;
    }
    using T = typename Elem<DT_OUT>::T;
    const T ql = Elem<DT_OUT>::put(lo), qh = Elem<DT_OUT>::put(hi), qf = Elem<DT_OUT>::put(fill);
    aux[0] = Elem<DT_OUT>::get(&ql, 0);
    aux[1] = Elem<DT_OUT>::get(&qh, 0);
    aux[2] = Elem<DT_OUT>::get(&qf, 0);
    aux[3] = bad ? 1.0f : 0.0f;
}

template <int DT_OUT, int C>
__global__ __launch_bounds__(kBlock) void upload_fill(VolDesc dst, int32_t groups_x,
                                                      const float* aux) {
    if (aux[3] == 0.0f) return;  // no non-finite voxel: nothing to replace
    using TO = typename Elem<DT_OUT>::T;
    constexpr int G = BrickGroup<C>::G;
    const int t = blockIdx.x;
    const int gx = t % groups_x;
    const int rest = t / groups_x;
    const int by = rest % dst.nby, bz = rest / dst.nby;
    const int bx0 = gx * G;
    const int nb = min(G, dst.nbx - bx0);
    TO* out = (TO*)dst.data + ((size_t)((size_t)bz * dst.nby + by) * dst.nbx + bx0) * dst.pitch;
    const TO fill = Elem<DT_OUT>::put(aux[2]);
    for (uint32_t e = threadIdx.x; e < (uint32_t)nb * dst.pitch; e += kBlock) {
        const float v = Elem<DT_OUT>::get(out, e);
        if (v != v) out[e] = fill;
    }
}

template <int DT_IN, int DT_OUT, int C>
static void upload_launch(const svr_cube_view& c, const VolDesc& d, float* aux, float nan_fill,
                          hipStream_t stream) {
    using TI = typename Elem<DT_IN>::T;
    const bool contig = c.sx == 0 && c.sy == 0 && c.sz == 0;
    const int64_t sx = contig ? 1 : c.sx;
    const int64_t sy = contig ? (int64_t)c.nx : c.sy;
    const int64_t sz = contig ? (int64_t)c.nx * c.ny : c.sz;
    const int groups_x = (d.nbx + BrickGroup<C>::G - 1) / BrickGroup<C>::G;
    const int nblocks = groups_x * d.nby * d.nbz;
    uint32_t* slots = reinterpret_cast<uint32_t*>(aux + 4);
    hipLaunchKernelGGL(upload_init, dim3(1), dim3(kBlock), 0, stream, slots);
    // 16-byte source loads need 16-byte aligned rows
    constexpr int VI = Vec16<TI>::N;
    const int vec_in = contig && c.nx % VI == 0 &&
                       (reinterpret_cast<uintptr_t>(c.data) & 15) == 0;
    if (contig)
        hipLaunchKernelGGL((brick_group_kernel<DT_IN, DT_OUT, C, true>), dim3(nblocks),
                           dim3(kBlock), 0, stream, (const TI*)c.data, sx, sy, sz, d, groups_x,
                           nblocks, vec_in, slots);
    else
        hipLaunchKernelGGL((brick_group_kernel<DT_IN, DT_OUT, C, false>), dim3(nblocks),
                           dim3(kBlock), 0, stream, (const TI*)c.data, sx, sy, sz, d, groups_x,
                           nblocks, 0, slots);
    hipLaunchKernelGGL(upload_final<DT_OUT>, dim3(1), dim3(kWave), 0, stream, aux, nan_fill);
    hipLaunchKernelGGL((upload_fill<DT_OUT, C>), dim3(nblocks), dim3(kBlock), 0, stream, d,
                       groups_x, (const float*)aux);
}

template <int DT_IN, int DT_OUT>
static void upload_launch_c(const svr_cube_view& c, const VolDesc& d, float* aux,
                            float nan_fill, hipStream_t stream) {
    if (d.brick == 16) upload_launch<DT_IN, DT_OUT, 16>(c, d, aux, nan_fill, stream);
    else upload_launch<DT_IN, DT_OUT, 8>(c, d, aux, nan_fill, stream);
}

template <int DT_IN>
static void upload_launch_in(const svr_cube_view& c, const VolDesc& d, float* aux,
                             float nan_fill, hipStream_t stream) {
    if (d.dtype == SVR_F16) upload_launch_c<DT_IN, SVR_F16>(c, d, aux, nan_fill, stream);
    else if (d.dtype == SVR_BF16) upload_launch_c<DT_IN, SVR_BF16>(c, d, aux, nan_fill, stream);
    else upload_launch_c<DT_IN, SVR_F32>(c, d, aux, nan_fill, stream);
}

svr_status launch_upload(const svr_cube_view& c, const VolDesc& d, float* aux, float nan_fill,
                         hipStream_t stream) {
    // at most one workgroup per brick, and bricks number below 2^24 (checked at creation)
    if (c.dtype == SVR_F16) upload_launch_in<SVR_F16>(c, d, aux, nan_fill, stream);
    else if (c.dtype == SVR_BF16) upload_launch_in<SVR_BF16>(c, d, aux, nan_fill, stream);
    else upload_launch_in<SVR_F32>(c, d, aux, nan_fill, stream);
    return hip_fail(hipGetLastError(), "upload launch");
}

// Bricked storage -> C-contiguous [z][y][x] of the storage type.
template <int DT, int C>
__global__ __launch_bounds__(kBlock) void export_kernel(VolDesc v, typename Elem<DT>::T* out) {
    constexpr int SH = C == 8 ? 3 : 4;
    using T = typename Elem<DT>::T;
    const uint32_t x = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t y = blockIdx.y, z = blockIdx.z;
    if (x >= (uint32_t)v.nx) return;
    const uint32_t b = ((z >> SH) * (uint32_t)v.nby + (y >> SH)) * (uint32_t)v.nbx + (x >> SH);
    const uint32_t loc = brick_loc<DT, C>(x & (C - 1), y & (C - 1), z & (C - 1));
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

// ------------------------------------------------------------ allocation-free min/max
// svr_minmax_noalloc keeps the per-workgroup partials of the reduction in this file-scope
// device array instead of a buffer from hipMalloc.  Every GPU the library runs on holds its
// own copy until the process ends.  In host code the name `scratch` is only a stand-in for
// the symbol: its device address is looked up once per device, with that device current,
// and only that address is handed to kernels.  The reduction never launches more than
// kMinmaxMaxBlocks workgroups, each writing its own partial before the final kernel reads
// it, so nothing in the array has to start at zero.  Calls that overlap on one GPU share
// the array and race.
constexpr int kMaxDevices = 64;
__device__ __align__(256) float scratch[3 * kMinmaxMaxBlocks];
static float* g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

static svr_status scratch_ptr(float** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "svr_minmax_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("svr_minmax_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
        return SVR_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "svr_minmax_noalloc: hipGetSymbolAddress");
        g_scratch[dev] = static_cast<float*>(p);
    }
    *ptr = g_scratch[dev];
    return SVR_OK;
}

svr_status launch_minmax_noalloc(const svr_cube_view& c, float* out, hipStream_t stream) {
    int64_t nx, nrows, ny, sx, sy, sz;
    dim3 grid;
    minmax_grid(c, nx, nrows, ny, sx, sy, sz, grid);
    const uint64_t parts = (uint64_t)grid.x * grid.y;
    if (3 * parts > sizeof(scratch) / sizeof(float)) {
        set_error("svr_minmax_noalloc: %llu partials exceed the %d the scratch array holds",
                  (unsigned long long)parts, kMinmaxMaxBlocks);
        return SVR_EINVAL;
    }
    float* partial = nullptr;
    svr_status st = scratch_ptr(&partial);
    if (st) return st;
    return launch_minmax(c, partial, out, 1, SVR_F32, NAN, stream);
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
