// Internal declarations shared by the HIP translation units of libsvr (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "svr.h"

namespace svr {

constexpr int kWave = 64;
constexpr int kTile = 16;            // image tile of one 256-lane workgroup (16 x 16 pixels)
constexpr int kBlock = 256;
constexpr int kCkptEvery = 32;       // samples between stored ray states (adjoint)

// Device view of a bricked volume.  Brick (bx, by, bz) holds voxels [C*b, C*b + C] per axis
// (C + 1 = E stored per axis; the last layer is the apron = first layer of the next brick,
// or a replica of the cube's last voxel); brick_index = (bz * nby + by) * nbx + bx.
//   float32: voxel (lx, ly, lz) of a brick sits at brick_index * pitch + (lz * E + ly) * E + lx.
//   16-bit:  y-pairs.  Pair (lx, ly, lz), ly < C, holds voxels (lx, ly, lz) and (lx, ly + 1, lz)
//            as two consecutive elements at brick_index * pitch + 2 ((lz * C + ly) * E + lx),
//            so one 8-byte load returns the four corners (x, x + 1) x (y, y + 1) of a cell face.
struct VolDesc {
    const void* data;
    int32_t nx, ny, nz;
    int32_t nbx, nby, nbz;
    int32_t dtype;
    int32_t brick;        // C
    uint32_t pitch;       // elements per brick (stored elements rounded up to 64)
    const float* clim;    // device: [finite min, finite max] of the stored values
};

// Stored elements of one brick: E^3 for float32, E C E pairs for 16-bit storage.
__host__ __device__ constexpr int brick_elems(int dtype, int C) {
    return dtype == SVR_F32 ? (C + 1) * (C + 1) * (C + 1) : 2 * (C + 1) * C * (C + 1);
}

// In-brick element offset of voxel (lx, ly, lz), ly < C for 16-bit storage (the first element
// of its pair; the pair of ly - 1 holds it too).
template <int DT, int C>
__host__ __device__ __forceinline__ uint32_t brick_loc(uint32_t lx, uint32_t ly, uint32_t lz) {
    constexpr uint32_t E = C + 1;
    return DT == SVR_F32 ? (lz * E + ly) * E + lx : 2u * ((lz * C + ly) * E + lx);
}

// Element offset of voxel cell (ix, iy, iz) in bricked storage: brick index (bz * nby + by)
// * nbx + bx times the pitch, plus the in-brick offset.  Coordinates, brick counts and the
// pitch are below 2^24 (checked at volume creation), which lets the device use 24-bit
// multiplies; the total is below 2^32.
template <int DT, int C>
__host__ __device__ __forceinline__ uint32_t cell_offset(uint32_t ix, uint32_t iy, uint32_t iz,
                                                         uint32_t nbx, uint32_t nby,
                                                         uint32_t pitch) {
    constexpr int SH = C == 8 ? 3 : 4;
    __builtin_assume(ix <= 0xffffffu);
    __builtin_assume(iy <= 0xffffffu);
    __builtin_assume(iz <= 0xffffffu);
    uint32_t b = (iz >> SH) * nby + (iy >> SH);
    __builtin_assume(b <= 0xffffffu);
    b = b * nbx + (ix >> SH);
    __builtin_assume(b <= 0xffffffu);
    return b * pitch + brick_loc<DT, C>(ix & (C - 1), iy & (C - 1), iz & (C - 1));
}

// Largest element offset, from a cell's first element, that a trilinear fetch reads: the
// corner (x + 1, y + 1, z + 1) for float32, the last element of the z + 1 pair face for
// 16-bit storage.
template <int DT, int C>
__host__ __device__ constexpr uint32_t corner_span() {
    return DT == SVR_F32 ? (uint32_t)((C + 1) * (C + 1) + (C + 1) + 1)
                         : (uint32_t)(2 * C * (C + 1) + 3);
}

// Brick grid and pitch of a volume of nx x ny x nz voxels (data and clim left null).
inline VolDesc make_voldesc(int32_t nx, int32_t ny, int32_t nz, int32_t dtype, int32_t brick) {
    VolDesc d{};
    d.nx = nx;
    d.ny = ny;
    d.nz = nz;
    d.nbx = (nx + brick - 1) / brick;
    d.nby = (ny + brick - 1) / brick;
    d.nbz = (nz + brick - 1) / brick;
    d.dtype = dtype;
    d.brick = brick;
    d.pitch = (uint32_t)((brick_elems(dtype, brick) + 63) / 64 * 64);
    return d;
}

// Streaming accesses for data a kernel reads or writes once: the non-temporal hint keeps them
// from displacing cached lines that other workgroups still use.  Measured: moment-map reads
// 7% faster, smoothing writes 1-2%; line-ratio reads and stores slower on small windows that
// later launches read again from the caches (kept plain), upload stores unchanged and upload
// reads 13% slower (neighbouring brick groups re-read each slab's halo rows from the caches);
// the ray-march's corner loads 1.7-3x slower (neighbouring rays share cached cells).
template <class T>
__device__ __forceinline__ T load_nt(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void store_nt(T v, T* p) {
    __builtin_nontemporal_store(v, p);
}

// Element loaders: stored type -> float32.
template <int DT> struct Elem;
template <> struct Elem<SVR_F32> {
    using T = float;
    static __device__ __forceinline__ float get(const T* p, uint32_t i) { return p[i]; }
    static __device__ __forceinline__ T put(float v) { return v; }
};
template <> struct Elem<SVR_F16> {
    using T = _Float16;
    static __device__ __forceinline__ float get(const T* p, uint32_t i) { return (float)p[i]; }
    // The float32 value rounded to nearest even.  The empty asm hides where v came from, so
    // the compiler cannot fold the FMA that produced it into a mixed-precision FMA that rounds
    // the exact result to half once: which of the two roundings a store got would then depend
    // on the code around it (one half ulp apart at ties).
    static __device__ __forceinline__ T put(float v) {
        asm("" : "+v"(v));
        return (_Float16)v;
    }
};
template <> struct Elem<SVR_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ float get(const T* p, uint32_t i) {
        return __uint_as_float(((uint32_t)p[i]) << 16);
    }
    static __device__ __forceinline__ T put(float v) {  // round to nearest even; NaN stays NaN
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x40u);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (T)(u >> 16);
    }
};

__device__ __forceinline__ float med3(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// True when the predicate holds on any lane of the wave (the same answer on every lane).
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// True when p is a multiple of `bytes` (the kernels load and store 16-byte RGBA texels and
// tables, and the split MIP renders combine 8-byte keys in the output).
inline bool aligned_to(const void* p, size_t bytes) {
    return (reinterpret_cast<uintptr_t>(p) % bytes) == 0;
}

// Workgroup b -> tile index so that each XCD (workgroups are dealt round-robin over the
// 8 XCDs) owns one contiguous run of tiles and its L2 sees neighbouring rays.
__host__ __device__ __forceinline__ int xcd_tile(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7, x = b & 7, s = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}

// Workgroup b -> tile index for work that varies from tile to tile (rays of different
// lengths).  Contiguous runs of kXcdRun tiles are dealt to the XCDs in turn, so each XCD owns
// every eighth run: spread over the whole image, which balances the XCDs' work (one band per
// XCD, as xcd_tile gives, leaves the XCDs whose bands miss the volume idle), while its L2
// still sees runs of neighbouring rays.  The last, incomplete round of 8 runs is split as
// xcd_tile splits a grid.
constexpr int kXcdRun = 4;
__host__ __device__ __forceinline__ int xcd_run_tile(int b, int nblocks) {
    const int full = nblocks / (8 * kXcdRun) * (8 * kXcdRun);
    if (b >= full) return full + xcd_tile(b - full, nblocks - full);
    const int x = b & 7, s = b >> 3;
    return ((s / kXcdRun) * 8 + x) * kXcdRun + s % kXcdRun;
}

// Ray of one pixel and its entry into the box [-0.5, n-0.5]^3, in double precision with
// every operation rounded separately (no contraction), so the entry point and the sample
// count match an IEEE double evaluation of the same formulas.  Returns the sample count
// (0 on a miss), the first sample position q0 and the per-sample step dq in double (sample
// k sits at q0 + k dq; positions reach ~1e3 voxels, where float spacing is ~1e-4 voxel,
// too coarse for trilinear weights near steep gradients), and both rounded to float for
// the normalised locations loc = (p + 0.5)/n that only colour the result.
struct RaySeg {
    double q0[3];
    double dq[3];
    float p0[3];
    float step[3];
    int32_t n;
};

__device__ inline RaySeg ray_segment(const svr_camera& c, int px, int py, int nx, int ny,
                                     int nz, float dtf) {
#pragma clang fp contract(off)
    // a miss keeps n = 0 and a valid point: lanes without samples still run the (uniform)
    // march loop and fetch at the volume origin
    RaySeg r;
    r.n = 0;
    r.q0[0] = r.q0[1] = r.q0[2] = 0.0;
    r.dq[0] = r.dq[1] = r.dq[2] = 0.0;
    r.p0[0] = r.p0[1] = r.p0[2] = 0.0f;
    r.step[0] = r.step[1] = r.step[2] = 0.0f;
    const double u = 2.0 * ((double)px + 0.5) / (double)c.width - 1.0;
    const double v = 2.0 * ((double)py + 0.5) / (double)c.height - 1.0;
    double o[3], d[3];
    for (int a = 0; a < 3; ++a) {
        if (c.type == 0) {
            o[a] = (double)c.eye[a] + u * (double)c.U[a] + v * (double)c.V[a];
            d[a] = (double)c.W[a];
        } else {
            o[a] = (double)c.eye[a];
            d[a] = (double)c.W[a] + u * (double)c.U[a] + v * (double)c.V[a];
        }
    }
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] = d[0] / len;
    d[1] = d[1] / len;
    d[2] = d[2] / len;
    if (!(isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]))) return r;
    const int n[3] = {nx, ny, nz};
    double tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double lo = -0.5, hi = (double)n[a] - 0.5;
        if (d[a] == 0.0) {
            if (o[a] < lo || o[a] > hi) return r;
            continue;
        }
        double ta = (lo - o[a]) / d[a];
        double tb = (hi - o[a]) / d[a];
        if (ta > tb) { const double t = ta; ta = tb; tb = t; }
        if (ta > tn) tn = ta;
        if (tb < tf) tf = tb;
    }
    if (tn < 0.0) tn = 0.0;
    if (!(tf > tn)) return r;
    const double dt = (double)dtf;
    r.n = (int32_t)ceil((tf - tn) / dt);
    for (int a = 0; a < 3; ++a) {
        r.q0[a] = o[a] + tn * d[a];
        r.dq[a] = dt * d[a];
        r.p0[a] = (float)r.q0[a];
        r.step[a] = (float)r.dq[a];
    }
    return r;
}

// One step of the normalised front-to-back compositing of Alg. AVIP0 (Eq. for alpha_2 and
// the colour/alpha update): a2 = k op (1 - a1), al = max(a1 + a2, minVal), colour
// c a1/al + c_s a2/al.  The colour update is evaluated as c + (c_s a2 - c (al - a1))/al,
// the same value in exact arithmetic, which leaves c exactly unchanged where a sample adds
// no opacity (a2 = 0, al = a1); the plain form would multiply c by a rounded a1 (1/al)
// ~ 1 +- 1 ulp on each such sample.  An inactive step (active = false) adds no opacity and
// keeps alpha, so it changes nothing.  Contraction is off so that every caller rounds
// a1 + a2 the same way.  Returns the new alpha.
struct Rgba {
    float r, g, b, a;
};

__device__ __forceinline__ float composite(Rgba& t, float cr, float cg, float cb, float op,
                                           float kw, float minv, bool active) {
#pragma clang fp contract(off)
    const float a1 = t.a;
    const float a2 = active ? kw * op * (1.0f - a1) : 0.0f;
    const float al0 = fmaxf(a1 + a2, minv);  // >= minv > 0
    const float al = active ? al0 : a1;
    const float ri = rcp(al0);
    const float w2 = a2 * ri, wd = (al - a1) * ri;
    t.r = fmaf(cr, w2, fmaf(-t.r, wd, t.r));
    t.g = fmaf(cg, w2, fmaf(-t.g, wd, t.g));
    t.b = fmaf(cb, w2, fmaf(-t.b, wd, t.b));
    t.a = al;
    return al;
}

// Colour/opacity table in LDS: the n entries followed by a copy of the last one, so the
// lookup needs no index clamp.
__device__ __forceinline__ void stage_table(float4* dst, const float4* src, int n) {
    for (int i = (int)threadIdx.x; i <= n; i += (int)blockDim.x) dst[i] = src[i < n ? i : n - 1];
}

// Table lookup: n RGBA entries at j/(n-1), linear interpolation; s in [0, 1], nm1 = n - 1.
// x = s (n-1) lies in [0, n-1]: interval j = trunc(x), weight f = x - j (exact).  At s = 1
// this reads entry n-1 with weight 1 - 0 and its copy with weight 0.
__device__ __forceinline__ float4 table(const float4* L, float nm1, float s) {
    const float x = s * nm1;
    const uint32_t j = (uint32_t)x;
    const float f = __builtin_amdgcn_fractf(x);
    const float4 a = L[j], b = L[j + 1];
    return make_float4(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y),
                       fmaf(f, b.z - a.z, a.z), fmaf(f, b.w - a.w, a.w));
}

// Host side helpers --------------------------------------------------------------------
// Byte offset past the end of every storage addressed with 32-bit offsets: buffer loads
// there return 0 without a memory access (the out-of-range reuse loads of the sampler).
constexpr uint32_t kPastStorage = 0xfffff000u;

// True when a volume's bricked storage is addressed with 64-bit offsets: storage that
// reaches kPastStorage bytes (so that 32-bit offsets from kPastStorage on always lie past
// its end).
inline bool wide_volume(const VolDesc& d) {
    const uint64_t esize = d.dtype == SVR_F32 ? 4 : 2;
    return (uint64_t)d.nbx * d.nby * d.nbz * d.pitch * esize > (uint64_t)kPastStorage;
}

void set_error(const char* fmt, ...);
svr_status hip_fail(hipError_t e, const char* what);

}  // namespace svr

// The opaque handles of the C ABI.
struct svr_volume {
    svr::VolDesc d;
    void* mem;          // bricked storage
    float* aux;         // clim[2], fill[1], partial reductions
    int64_t bytes;
    int device;
};
