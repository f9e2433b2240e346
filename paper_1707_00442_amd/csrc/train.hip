// Differentiable AVIP0 with a piecewise-linear RGBA transfer function, and its adjoint.
//
// Forward (train_fwd_kernel): the AVIP0 ray-march of the render path with colour = tf(s).rgb
// and opacity weight k * tf(s).a; every 32 samples the ray state (C, A) before the sample
// is stored, and at the end the number of composited samples K.  The image equals the
// plain render with opacity_from_lut = 1.
//
// Backward (train_bwd_kernel): see the kernel.  Per-sample states live in registers for one
// 8-sample sub-segment at a time (two-level replay from the 32-sample checkpoints).
#include "sampler.h"

namespace svr {

constexpr int kTrainMaxTf = 256;

struct TrainArgs {
    VolDesc v;
    svr_camera cam;
    const float4* tf;
    int32_t tf_n;
    svr_params p;
    float4* out;
    int32_t* kcount;
    float4* ckpt;
    int64_t nrays;
    int32_t nseg, tiles_x, nblocks;
    const float4* grad;
    float* grad_tf;
    float* grad_vox;
};

// One step of the compositing of Alg. AVIP0, the same function as the render path.
using AvipState = Rgba;

__device__ __forceinline__ void avip_step(AvipState& t, float4 c, float kw, float minv) {
    composite(t, c.x, c.y, c.z, c.w, kw, minv, true);
}

template <int DT, int C>
__global__ __launch_bounds__(kBlock) void train_fwd_kernel(const TrainArgs a) {
    __shared__ float4 s_tf[kTrainMaxTf + 1];
    stage_table(s_tf, a.tf, a.tf_n);
    __syncthreads();
    const int t = xcd_run_tile((int)blockIdx.x, a.nblocks);
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int px = tx * kTile + (w & 1) * 8 + (l & 7);
    const int py = ty * kTile + (w >> 1) * 8 + (l >> 3);
    const int64_t rid = (int64_t)t * kBlock + threadIdx.x;
    if (px >= a.cam.width || py >= a.cam.height) {
        a.kcount[rid] = 0;
        return;
    }
    float lo = a.p.clim_lo, hi = a.p.clim_hi;
    if (!(hi > lo)) {
        lo = a.v.clim[0];
        hi = a.v.clim[1];
    }
    const float inv = hi > lo ? 1.0f / (hi - lo) : 0.0f;
    const RaySeg r = ray_segment(a.cam, px, py, a.v.nx, a.v.ny, a.v.nz, a.p.dt);
    const Sampler<DT, C, true> smp(a.v);
    AvipState st{0.0f, 0.0f, 0.0f, 0.0f};
    const float kw = a.p.k, minv = a.p.min_val, ert = a.p.ert;
    int K = 0;
    float kf = 0.0f;
    for (int k = 0; k < r.n; ++k, kf += 1.0f) {
        if ((k & (kCkptEvery - 1)) == 0)
            a.ckpt[(int64_t)(k / kCkptEvery) * a.nrays + rid] = make_float4(st.r, st.g, st.b, st.a);
        const double kd = (double)kf;
        const float v = smp(fma(kd, r.dq[0], r.q0[0]), fma(kd, r.dq[1], r.q0[1]),
                            fma(kd, r.dq[2], r.q0[2]));
        const float s = __saturatef((v - lo) * inv);
        avip_step(st, table(s_tf, (float)(a.tf_n - 1), s), kw, minv);
        ++K;
        if (st.a > ert) break;
    }
    a.kcount[rid] = K;
    a.out[(size_t)py * a.cam.width + px] = make_float4(st.r, st.g, st.b, st.a);
}

// Per-lane accumulators flushed only when their key changes: consecutive samples of a ray
// usually share the table interval and the voxel cell, so most atomic adds are merged.
struct TfAccum {
    int j = -1;
    float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    __device__ __forceinline__ void flush(float* s_gtf) {
        if (j < 0) return;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (v[q] != 0.0f) atomicAdd(&s_gtf[4 * j + q], v[q]);
    }
    __device__ __forceinline__ void add(float* s_gtf, int jj, const float (&e)[8]) {
        if (jj != j) {
            flush(s_gtf);
            j = jj;
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = e[q];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] += e[q];
        }
    }
};

// Table-gradient window of one lane: entries [base, base + 8) held in registers.  A ray's
// samples mostly stay within a few neighbouring table intervals (the noise floor of the
// cube), so the window takes most updates with plain adds; an interval outside it goes to
// the flush-on-change accumulator.  The window is placed around the first interval seen.
// Table entries in the window: 8 measured fastest (backward at 1024^2 through 256^3: 2.77 ms;
// 6 entries 2.85 ms, 4 entries 3.07 ms, more intervals then going to the LDS accumulator).
constexpr int kTfWin = 8;
struct TfWindow {
    int base = -1;
    float w[kTfWin][4] = {};
    // entries j and j + 1 get weights 1 - f and f of gc; false if they are not both inside
    __device__ __forceinline__ bool add(int j, float f, const float (&gc)[4], int n) {
        if (base < 0) base = max(0, min(j - (kTfWin / 2 - 1), n - kTfWin));
        const int rel = j - base;
        if (rel < 0 || rel > kTfWin - 2) return false;
        const float wj = 1.0f - f;
#pragma unroll
        for (int q = 0; q < kTfWin; ++q) {
            const float wq = q == rel ? wj : (q == rel + 1 ? f : 0.0f);
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) w[q][ch] = fmaf(wq, gc[ch], w[q][ch]);
        }
        return true;
    }
    __device__ __forceinline__ void flush(float* s_gtf, int n) const {
        if (base < 0) return;
#pragma unroll
        for (int q = 0; q < kTfWin; ++q)
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                if (base + q < n && w[q][ch] != 0.0f) atomicAdd(&s_gtf[4 * (base + q) + ch], w[q][ch]);
    }
};

struct VoxAccum {
    int64_t key = -1;  // linear index of the cell's first corner
    uint32_t i0 = 0, j0 = 0, l0 = 0;
    float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // Corner q of the cell is (dx, dy, dz) = (q & 1, (q >> 1) & 1, q >> 2).  Neighbouring
    // rays share corners, so lane l (pixel (l mod 8, l / 8) of the wave's 8 x 8 block)
    // issues corner (q + rot) mod 8 at step q with rot = (l + 3 (l / 8)) mod 8: the eight
    // lanes of a pixel row, of a pixel column and of every 2 x 2 block get distinct
    // rotations, so the lanes of one atomic instruction mostly target distinct addresses
    // (atomics to one address within an instruction are serialised).  add(q, value)
    // receives corner q, for the corners set in mask.
    template <class Add>
    __device__ __forceinline__ void each_corner(unsigned mask, Add&& add) const {
        const int l = (int)(threadIdx.x & 63);
        const int rot = (l + 3 * (l >> 3)) & 7;
        // rotate (v[0..7]) left by rot with three conditional stages
        float r[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = v[q];
        if (rot & 1) {
            const float t0 = r[0];
#pragma unroll
            for (int q = 0; q < 7; ++q) r[q] = r[q + 1];
            r[7] = t0;
        }
        if (rot & 2) {
            const float t0 = r[0], t1 = r[1];
#pragma unroll
            for (int q = 0; q < 6; ++q) r[q] = r[q + 2];
            r[6] = t0;
            r[7] = t1;
        }
        if (rot & 4) {
            const float t0 = r[0], t1 = r[1], t2 = r[2], t3 = r[3];
            r[0] = r[4]; r[1] = r[5]; r[2] = r[6]; r[3] = r[7];
            r[4] = t0; r[5] = t1; r[6] = t2; r[7] = t3;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int cq = (q + rot) & 7;
            if ((mask >> cq) & 1u) add(cq, r[q]);
        }
    }
    // add the pending corners in mask to the global gradient (nx * ny * nz, x fastest)
    __device__ __forceinline__ void flush(float* G, uint32_t nx, uint32_t ny, uint32_t nz,
                                          unsigned mask = 0xffu) {
        if (key < 0) return;
        const uint32_t i1 = min(i0 + 1, nx - 1), j1 = min(j0 + 1, ny - 1), l1 = min(l0 + 1, nz - 1);
        const int64_t dxo = (int64_t)i1 - i0;
        const int64_t dyo = ((int64_t)j1 - j0) * nx;
        const int64_t dzo = ((int64_t)l1 - l0) * nx * ny;
        float* base = G + key;
        each_corner(mask, [&](int cq, float x) {
            unsafeAtomicAdd(base + ((cq & 1) ? dxo : 0) + ((cq & 2) ? dyo : 0) +
                            ((cq & 4) ? dzo : 0), x);
        });
        key = -1;
    }
    // add the pending corners in mask to the workgroup's box of voxels [b0, b0 + bn)
    // (x fastest); a cell outside the box goes to the global gradient instead
    __device__ __forceinline__ void flush_box(float* box, const int (&b0)[3], const int (&bn)[3],
                                              float* G, uint32_t nx, uint32_t ny, uint32_t nz,
                                              unsigned mask = 0xffu) {
        if (key < 0) return;
        const uint32_t i1 = min(i0 + 1, nx - 1), j1 = min(j0 + 1, ny - 1), l1 = min(l0 + 1, nz - 1);
        const int x0 = (int)i0 - b0[0], y0 = (int)j0 - b0[1], z0 = (int)l0 - b0[2];
        const int x1 = (int)i1 - b0[0], y1 = (int)j1 - b0[1], z1 = (int)l1 - b0[2];
        if (x0 < 0 || y0 < 0 || z0 < 0 || x1 >= bn[0] || y1 >= bn[1] || z1 >= bn[2]) {
            flush(G, nx, ny, nz, mask);
            return;
        }
        const int dxo = x1 - x0, dyo = (y1 - y0) * bn[0], dzo = (z1 - z0) * bn[0] * bn[1];
        float* base = box + (z0 * bn[1] + y0) * bn[0] + x0;
        each_corner(mask, [&](int cq, float x) {
            atomicAdd(base + ((cq & 1) ? dxo : 0) + ((cq & 2) ? dyo : 0) + ((cq & 4) ? dzo : 0), x);
        });
        key = -1;
    }
};

constexpr int kSub = 4;  // samples per sub-segment (held in registers)
static_assert(kCkptEvery % kSub == 0, "checkpoint segments split into sub-segments");
constexpr int kBox = 4096;  // voxels of the workgroup's LDS gradient box (16 KB, <= 2^13)
// LDS copies of the table gradient: lane t adds into copy t mod ncopy, so lanes whose rays
// sit in the same table interval mostly hit different copies; copies are 4 n + 1 floats
// apart, which puts one entry's copies in different LDS banks.
constexpr int kGtfLds = 4096;
constexpr int kWaves = kBlock / 64;

// Minimum (first three) and maximum (last three) of six per-lane integers over the
// workgroup; every thread receives the result.  The caller separates two calls by a barrier.
__device__ __forceinline__ void wg_box(int (&b)[6], int (*s_red)[kWaves]) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
        for (int o = 32; o > 0; o >>= 1) {
            const int y = __shfl_xor(b[i], o);
            b[i] = i < 3 ? min(b[i], y) : max(b[i], y);
        }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 6; ++i) s_red[i][threadIdx.x >> 6] = b[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        int m = s_red[i][0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) m = i < 3 ? min(m, s_red[i][w]) : max(m, s_red[i][w]);
        b[i] = __builtin_amdgcn_readfirstlane(m);  // uniform: keep it in scalar registers
    }
}

// Backward: the workgroup layout and ray ids of the forward pass.  The workgroup walks
// checkpoint segments from the last to the first, segment index by segment index (each
// ray's segments start at its own first sample).  Within a segment a ray is replayed once
// from its stored state to find the states at its sub-segment starts; each sub-segment,
// last first, is replayed again into registers (state before each sample and its s) and
// then run through the reverse recurrence of the normalised compositing step.  Gradients
// of the table entries go to the workgroup's LDS copy (one global atomic per entry at the
// end), through a per-lane register window of eight entries where the samples fall inside
// it.  Gradients of the voxels go to the eight trilinear corners: into an LDS box that
// holds every cell the workgroup's rays visit in the segment when it fits (one global
// atomic per touched voxel per segment), else straight to global memory with hardware
// float atomics.
template <int DT, int C>
__global__ __launch_bounds__(kBlock) void train_bwd_kernel(const TrainArgs a) {
    __shared__ float4 s_tf[kTrainMaxTf + 1];
    __shared__ float s_gtf[kGtfLds];
    __shared__ float4 s_sub[kCkptEvery / kSub][kBlock];  // sub-segment start states
    __shared__ float s_box[kBox];
    __shared__ int s_red[6][kWaves];
    const int n = a.tf_n;
    const bool want_vox = a.grad_vox != nullptr;
    stage_table(s_tf, a.tf, n);
    const int gstride = 4 * n + 1;
    const int ncopy = min(16, kGtfLds / gstride);
    for (int i = threadIdx.x; i < kGtfLds; i += kBlock) s_gtf[i] = 0.0f;
    float* const my_gtf = s_gtf + (int)(threadIdx.x % (unsigned)ncopy) * gstride;
    if (want_vox)
        for (int i = threadIdx.x; i < kBox; i += kBlock) s_box[i] = 0.0f;
    __syncthreads();

    const int t = xcd_run_tile((int)blockIdx.x, a.nblocks);
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int px = tx * kTile + (w & 1) * 8 + (l & 7);
    const int py = ty * kTile + (w >> 1) * 8 + (l >> 3);
    const int64_t rid = (int64_t)t * kBlock + threadIdx.x;
    const bool inside = px < a.cam.width && py < a.cam.height;
    const int K = inside ? a.kcount[rid] : 0;
    float lo = a.p.clim_lo, hi = a.p.clim_hi;
    if (!(hi > lo)) {
        lo = a.v.clim[0];
        hi = a.v.clim[1];
    }
    const float inv = hi > lo ? 1.0f / (hi - lo) : 0.0f;
    const RaySeg r = ray_segment(a.cam, inside ? px : 0, inside ? py : 0, a.v.nx, a.v.ny,
                                 a.v.nz, a.p.dt);
    const Sampler<DT, C, true> smp(a.v);
    const float kw = a.p.k, minv = a.p.min_val;
    const float nm1 = (float)(n - 1);
    const float4 g = K > 0 ? a.grad[(size_t)py * a.cam.width + px] : make_float4(0, 0, 0, 0);
    float gr = g.x, gg = g.y, gb = g.z, ga = g.w;
    const uint32_t nx = (uint32_t)a.v.nx, ny = (uint32_t)a.v.ny, nz = (uint32_t)a.v.nz;
    const double xm = a.v.nx - 1, ym = a.v.ny - 1, zm = a.v.nz - 1;
    TfAccum tfa;
    TfWindow tfw;
    VoxAccum vxa;
    bool in_box = false;  // this segment's voxel gradients go to the LDS box
    int b0[3] = {0, 0, 0}, bn[3] = {0, 0, 0};
    // the clamped position of sample k (the forward pass's fetch)
    auto pos = [&](int k, double (&p)[3]) {
        const double kd = (double)k;
        p[0] = fmin(fmax(fma(kd, r.dq[0], r.q0[0]), 0.0), xm);
        p[1] = fmin(fmax(fma(kd, r.dq[1], r.q0[1]), 0.0), ym);
        p[2] = fmin(fmax(fma(kd, r.dq[2], r.q0[2]), 0.0), zm);
    };
    // normalised value of sample k (filter none)
    auto sample_s = [&](int k) -> float {
        const double kd = (double)k;
        const float v = smp(fma(kd, r.dq[0], r.q0[0]), fma(kd, r.dq[1], r.q0[1]),
                            fma(kd, r.dq[2], r.q0[2]));
        return __saturatef((v - lo) * inv);
    };
    auto vox_flush = [&](unsigned mask) {
        if (in_box)
            vxa.flush_box(s_box, b0, bn, a.grad_vox, nx, ny, nz, mask);
        else
            vxa.flush(a.grad_vox, nx, ny, nz, mask);
    };
    // reverse step for sample k with state-before S0 and value s
    auto reverse = [&](int k, const float4 S0, float s) {
        const float4 c = table(s_tf, nm1, s);
        const float a_ = kw * c.w;
        const float a1 = S0.w;
        const float a2 = a_ * (1.0f - a1);
        const float sum = __fadd_rn(a1, a2);  // rounded as in composite()
        const bool act = sum >= minv;
        const float al = fmaxf(sum, minv);
        const float ri = rcp(al);
        const float w1 = a1 * ri, w2 = a2 * ri, wd = (al - a1) * ri;
        const float C1r = fmaf(c.x, w2, fmaf(-S0.x, wd, S0.x));  // as composite()
        const float C1g = fmaf(c.y, w2, fmaf(-S0.y, wd, S0.y));
        const float C1b = fmaf(c.z, w2, fmaf(-S0.z, wd, S0.z));
        const float g_al = ga - (gr * C1r + gg * C1g + gb * C1b) * ri;
        const float g_a2 = (gr * c.x + gg * c.y + gb * c.z) * ri + (act ? g_al : 0.0f);
        const float g_a1 = (gr * S0.x + gg * S0.y + gb * S0.z) * ri + (act ? g_al : 0.0f) -
                           g_a2 * a_;
        const float gcr = gr * w2, gcg = gg * w2, gcb = gb * w2;
        const float gop = kw * g_a2 * (1.0f - a1);
        // table: interval j and weight f of the forward lookup (the entry weights)
        const float x = s * nm1;
        int j = (int)x;
        j = j > n - 2 ? n - 2 : j;
        const float f = x - (float)j;
        const float gcv[4] = {gcr, gcg, gcb, gop};
        if (!tfw.add(j, f, gcv, n)) {
            const float e[8] = {(1.0f - f) * gcr, (1.0f - f) * gcg, (1.0f - f) * gcb,
                                (1.0f - f) * gop, f * gcr, f * gcg, f * gcb, f * gop};
            tfa.add(my_gtf, j, e);
        }
        if (want_vox && s > 0.0f && s < 1.0f) {
            const float4 P0 = s_tf[j], P1 = s_tf[j + 1];
            const float gs = (gcr * (P1.x - P0.x) + gcg * (P1.y - P0.y) +
                              gcb * (P1.z - P0.z) + gop * (P1.w - P0.w)) * nm1;
            const float gv = gs * inv;
            // the cell and fractions of the forward fetch (double positions)
            double q[3];
            pos(k, q);
            const float fx = (float)__builtin_amdgcn_fract(q[0]);
            const float fy = (float)__builtin_amdgcn_fract(q[1]);
            const float fz = (float)__builtin_amdgcn_fract(q[2]);
            const uint32_t i0 = (uint32_t)q[0], j0 = (uint32_t)q[1], l0 = (uint32_t)q[2];
            const int64_t key = ((int64_t)l0 * ny + j0) * nx + i0;
            const float gx0 = gv * (1.0f - fx), gx1 = gv * fx;
            const float wy0z0 = (1.0f - fy) * (1.0f - fz), wy1z0 = fy * (1.0f - fz);
            const float wy0z1 = (1.0f - fy) * fz, wy1z1 = fy * fz;
            const float d8[8] = {gx0 * wy0z0, gx1 * wy0z0, gx0 * wy1z0, gx1 * wy1z0,
                                 gx0 * wy0z1, gx1 * wy0z1, gx0 * wy1z1, gx1 * wy1z1};
            if (key != vxa.key) {
                // A step to a face-adjacent cell keeps the four corners of the shared face
                // (axis bit b, +-1): only the corners left behind are flushed.  At the
                // upper volume edge both cells' corners map to the same clamped voxels.
                unsigned mask = 0xffu;
                int b = 0;
                if (vxa.key >= 0) {
                    const int di = (int)i0 - (int)vxa.i0, dj = (int)j0 - (int)vxa.j0;
                    const int dl = (int)l0 - (int)vxa.l0;
                    if (abs(di) + abs(dj) + abs(dl) == 1) {
                        b = di != 0 ? 1 : (dj != 0 ? 2 : 4);
                        const unsigned lower = b == 1 ? 0x55u : (b == 2 ? 0x33u : 0x0fu);
                        mask = di + dj + dl > 0 ? lower : (~lower & 0xffu);
                    }
                }
                vox_flush(mask);
                float nv[8];
#pragma unroll
                for (int q8 = 0; q8 < 8; ++q8) {
                    // new corner q8 continues old corner q8 ^ b when that one was kept (the
                    // three candidates are read first: a select between array elements
                    // would become a dynamic index and move the array to scratch memory)
                    const float o1 = vxa.v[q8 ^ 1], o2 = vxa.v[q8 ^ 2], o4 = vxa.v[q8 ^ 4];
                    const float ov = b == 1 ? o1 : (b == 2 ? o2 : o4);
                    const bool kept = b != 0 && !((mask >> (q8 ^ b)) & 1u);
                    nv[q8] = kept ? d8[q8] + ov : d8[q8];
                }
                vxa.key = key;
                vxa.i0 = i0;
                vxa.j0 = j0;
                vxa.l0 = l0;
#pragma unroll
                for (int q8 = 0; q8 < 8; ++q8) vxa.v[q8] = nv[q8];
            } else {
#pragma unroll
                for (int q8 = 0; q8 < 8; ++q8) vxa.v[q8] += d8[q8];
            }
        }
        gr *= w1;
        gg *= w1;
        gb *= w1;
        ga = g_a1;
    };
    // one sub-segment, last sample first: replay into registers, then reverse
    auto sub_segment = [&](int kb, int k1, Rgba st) {
        float4 S[kSub];
        float sv[kSub];
#pragma unroll
        for (int i = 0; i < kSub; ++i) {
            S[i] = make_float4(st.r, st.g, st.b, st.a);
            sv[i] = 0.0f;
            if (kb + i < k1) {
                sv[i] = sample_s(kb + i);
                avip_step(st, table(s_tf, nm1, sv[i]), kw, minv);
            }
        }
#pragma unroll
        for (int i = kSub - 1; i >= 0; --i)
            if (kb + i < k1) reverse(kb + i, S[i], sv[i]);
    };
    // segment count of the workgroup (lanes without samples have none)
    const int myseg = K > 0 ? (K - 1) / kCkptEvery : -1;
    int nb[6] = {0, 0, 0, myseg, 0, 0};
    wg_box(nb, s_red);
    for (int seg = nb[3]; seg >= 0; --seg) {
        const bool mine = seg <= myseg;
        const int k0 = seg * kCkptEvery;
        const int k1 = mine ? min(k0 + kCkptEvery, K) : k0;
        if (want_vox) {
            // cells of this segment: positions are monotone in k, so the first and the
            // last sample bound them; corners reach one further, up to n - 1
            int bb[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -1, -1, -1};
            if (mine) {
                double pa[3], pb[3];
                pos(k0, pa);
                pos(k1 - 1, pb);
                const int nmax[3] = {(int)nx - 1, (int)ny - 1, (int)nz - 1};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    bb[d] = (int)fmin(pa[d], pb[d]);
                    bb[3 + d] = min((int)fmax(pa[d], pb[d]) + 1, nmax[d]);
                }
            }
            __syncthreads();  // s_red of the previous reduction has been read
            wg_box(bb, s_red);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                b0[d] = bb[d];
                bn[d] = bb[3 + d] - bb[d] + 1;
            }
            in_box = bb[3] >= 0 &&
                     (int64_t)bn[0] * bn[1] * bn[2] <= (int64_t)kBox;
        }
        if (mine) {
            const float4 c0 = a.ckpt[(int64_t)seg * a.nrays + rid];
            // states at the sub-segment starts (LDS, one slot per lane)
            Rgba st{c0.x, c0.y, c0.z, c0.w};
            const int nsub = (k1 - k0 + kSub - 1) / kSub;
            for (int u = 0; u < nsub; ++u) {
                s_sub[u][threadIdx.x] = make_float4(st.r, st.g, st.b, st.a);
                if (u == nsub - 1) break;
                for (int k = k0 + u * kSub; k < k0 + (u + 1) * kSub; ++k)
                    avip_step(st, table(s_tf, nm1, sample_s(k)), kw, minv);
            }
            for (int u = nsub - 1; u >= 0; --u) {
                const float4 q = s_sub[u][threadIdx.x];
                sub_segment(k0 + u * kSub, k1, Rgba{q.x, q.y, q.z, q.w});
            }
            if (want_vox) vox_flush(0xffu);
        }
        if (in_box) {
            // the box to global memory, one atomic per touched voxel; the box is left zero.
            // Element e = (ez * bn1 + ey) * bn0 + ex; the quotients use reciprocal
            // multipliers m = floor((2^32 - 1) / d) + 1, exact for e, d <= 2^13 (kBox).
            __syncthreads();
            const uint32_t nxy = (uint32_t)(bn[0] * bn[1]), vol = nxy * (uint32_t)bn[2];
            const uint32_t m0 = 0xffffffffu / (uint32_t)bn[0] + 1u, m1 = 0xffffffffu / nxy + 1u;
            float* G0 = a.grad_vox + ((int64_t)b0[2] * ny + b0[1]) * nx + b0[0];
            const int64_t sxy = (int64_t)nx * ny;
            for (uint32_t e = threadIdx.x; e < vol; e += kBlock) {
                const float v = s_box[e];
                if (v != 0.0f) {
                    const uint32_t ez = nxy > 1 ? __umulhi(e, m1) : e;
                    const uint32_t rem = e - ez * nxy;
                    const uint32_t ey = bn[0] > 1 ? __umulhi(rem, m0) : rem;
                    const uint32_t ex = rem - ey * (uint32_t)bn[0];
                    unsafeAtomicAdd(G0 + (int64_t)ez * sxy + (int64_t)ey * nx + ex, v);
                    s_box[e] = 0.0f;
                }
            }
        }
    }
    tfa.flush(my_gtf);
    tfw.flush(my_gtf, n);
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * n; i += kBlock) {
        float v = 0.0f;
        for (int q = 0; q < ncopy; ++q) v += s_gtf[q * gstride + i];
        if (v != 0.0f) unsafeAtomicAdd(a.grad_tf + i, v);
    }
}

// ------------------------------------------------------------------------------- host side
svr_status check_camera(const svr_camera* c);
svr_status check_lut(const svr_lut* l);
svr_status check_params(const svr_params* p, const svr_volume* v);

static svr_status train_checks(const svr_volume* vol, const svr_camera* cam,
                               const svr_params* p) {
    if (!vol) {
        set_error("null volume");
        return SVR_EINVAL;
    }
    svr_status st = check_camera(cam);
    if (st) return st;
    if ((st = check_params(p, vol))) return st;
    if (p->mode != SVR_AVIP0 || p->filter != SVR_FILTER_NONE || p->box_arm != 0 ||
        p->ratio != 0 || p->opacity_from_lut != 1 || p->star_n != 0) {
        set_error("differentiable render: mode SVR_AVIP0, filter none, box_arm 0, ratio 0, "
                  "star_n 0, opacity_from_lut 1");
        return SVR_EINVAL;
    }
    return SVR_OK;
}

struct TrainGeom {
    int tiles_x, nblocks, nseg;
    int64_t nrays;
    size_t bytes;
};

static TrainGeom train_geom(const svr_volume* v, const svr_camera& cam, float dt) {
    TrainGeom g;
    g.tiles_x = (cam.width + kTile - 1) / kTile;
    g.nblocks = g.tiles_x * ((cam.height + kTile - 1) / kTile);
    g.nrays = (int64_t)g.nblocks * kBlock;
    const double diag = sqrt((double)v->d.nx * v->d.nx + (double)v->d.ny * v->d.ny +
                             (double)v->d.nz * v->d.nz);
    const int64_t maxn = (int64_t)ceil(diag / (double)dt) + 2;
    g.nseg = (int)((maxn + kCkptEvery - 1) / kCkptEvery);
    g.bytes = 256 + (size_t)g.nrays * sizeof(int32_t) + (size_t)g.nseg * g.nrays * sizeof(float4);
    return g;
}

template <int DT, int C>
static void train_launch(bool fwd, const TrainArgs& a, hipStream_t s) {
    if (fwd)
        hipLaunchKernelGGL((train_fwd_kernel<DT, C>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((train_bwd_kernel<DT, C>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
}

static void train_dispatch(bool fwd, int dtype, int brick, const TrainArgs& a, hipStream_t s) {
    if (brick == 16) {
        if (dtype == SVR_F16) train_launch<SVR_F16, 16>(fwd, a, s);
        else if (dtype == SVR_BF16) train_launch<SVR_BF16, 16>(fwd, a, s);
        else train_launch<SVR_F32, 16>(fwd, a, s);
    } else {
        if (dtype == SVR_F16) train_launch<SVR_F16, 8>(fwd, a, s);
        else if (dtype == SVR_BF16) train_launch<SVR_BF16, 8>(fwd, a, s);
        else train_launch<SVR_F32, 8>(fwd, a, s);
    }
}

}  // namespace svr

using namespace svr;

extern "C" {

svr_status svr_render_train_workspace(const svr_volume* vol, const svr_camera* cam,
                                      const svr_params* params, size_t* bytes) {
    svr_status st = train_checks(vol, cam, params);
    if (st) return st;
    if (!bytes) {
        set_error("null output");
        return SVR_EINVAL;
    }
    *bytes = train_geom(vol, *cam, params->dt).bytes;
    return SVR_OK;
}

svr_status svr_render_train(const svr_volume* vol, const svr_camera* cam, const svr_lut* tf,
                            const svr_params* params, float* rgba_out, void* workspace,
                            size_t workspace_bytes, void* stream) {
    svr_status st = train_checks(vol, cam, params);
    if (st) return st;
    if ((st = check_lut(tf))) return st;
    if (tf->n > kTrainMaxTf) {
        set_error("differentiable render: transfer function of %d > %d points", tf->n, kTrainMaxTf);
        return SVR_EINVAL;
    }
    if (!rgba_out || !workspace) {
        set_error("null output or workspace");
        return SVR_EINVAL;
    }
    if (!aligned_to(rgba_out, 16) || !aligned_to(workspace, 16)) {
        set_error("output or workspace not 16-byte aligned");
        return SVR_EINVAL;
    }
    const TrainGeom g = train_geom(vol, *cam, params->dt);
    if (workspace_bytes < g.bytes) {
        set_error("workspace %zu < %zu bytes", workspace_bytes, g.bytes);
        return SVR_ENOMEM;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    TrainArgs a{};
    a.v = vol->d;
    a.cam = *cam;
    a.tf = reinterpret_cast<const float4*>(tf->rgba);
    a.tf_n = tf->n;
    a.p = *params;
    a.out = reinterpret_cast<float4*>(rgba_out);
    a.kcount = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + 256);
    a.ckpt = reinterpret_cast<float4*>(static_cast<char*>(workspace) + 256 +
                                       (size_t)g.nrays * sizeof(int32_t));
    a.nrays = g.nrays;
    a.nseg = g.nseg;
    a.tiles_x = g.tiles_x;
    a.nblocks = g.nblocks;
    train_dispatch(true, vol->d.dtype, vol->d.brick, a, s);
    return hip_fail(hipGetLastError(), "train forward launch");
}

svr_status svr_render_backward(const svr_volume* vol, const svr_camera* cam, const svr_lut* tf,
                               const svr_params* params, const void* workspace,
                               size_t workspace_bytes, const float* grad_rgba,
                               float* grad_tf, float* grad_vox, void* stream) {
    svr_status st = train_checks(vol, cam, params);
    if (st) return st;
    if ((st = check_lut(tf))) return st;
    if (tf->n > kTrainMaxTf) {
        set_error("differentiable render: transfer function of %d > %d points", tf->n, kTrainMaxTf);
        return SVR_EINVAL;
    }
    if (!workspace || !grad_rgba || !grad_tf) {
        set_error("null workspace, grad_rgba or grad_tf");
        return SVR_EINVAL;
    }
    if (!aligned_to(workspace, 16) || !aligned_to(grad_rgba, 16) || !aligned_to(grad_tf, 4) ||
        !aligned_to(grad_vox, 4)) {
        set_error("workspace or grad_rgba not 16-byte aligned, or a gradient not 4-byte aligned");
        return SVR_EINVAL;
    }
    const TrainGeom g = train_geom(vol, *cam, params->dt);
    if (workspace_bytes < g.bytes) {
        set_error("workspace %zu < %zu bytes", workspace_bytes, g.bytes);
        return SVR_ENOMEM;
    }
    TrainArgs a{};
    a.v = vol->d;
    a.cam = *cam;
    a.tf = reinterpret_cast<const float4*>(tf->rgba);
    a.tf_n = tf->n;
    a.p = *params;
    a.kcount = reinterpret_cast<int32_t*>(static_cast<char*>(const_cast<void*>(workspace)) + 256);
    a.ckpt = reinterpret_cast<float4*>(static_cast<char*>(const_cast<void*>(workspace)) + 256 +
                                       (size_t)g.nrays * sizeof(int32_t));
    a.nrays = g.nrays;
    a.nseg = g.nseg;
    a.tiles_x = g.tiles_x;
    a.nblocks = g.nblocks;
    a.grad = reinterpret_cast<const float4*>(grad_rgba);
    a.grad_tf = grad_tf;
    a.grad_vox = grad_vox;
    train_dispatch(false, vol->d.dtype, vol->d.brick, a, static_cast<hipStream_t>(stream));
    return hip_fail(hipGetLastError(), "train backward launch");
}

}  // extern "C"
