// Batched rendering of many sub-cubes (each with its own camera and image) in one
// persistent launch.
//
// The host builds a work queue of (volume, tile) items, ordered by an estimate of their
// sample count (longest first), and a device table of per-volume descriptors.  A grid of
// persistent 256-lane workgroups drains the queue: one lane claims the next item with a
// global atomic counter, the workgroup renders that tile with the same per-ray code as
// svr_render (so every image is bit-identical to a single-image render), and loops until
// the queue is empty -- every workgroup exits once the counter passes the queue length.
// The pair (counter reset kernel, persistent kernel) is captured once into a HIP graph.
//
// The autotuner searches brick edge (8, 16) x tile shape (8x32, 16x16, 32x8 pixels: four
// 8x8 waves) x grid size (2, 4, 8 workgroups per CU) on the real batch: each candidate is
// timed as the median of three launches after a warm-up.  A brick edge other than that of
// the caller's volumes is tried on copies re-bricked by the library (the images do not
// depend on the brick edge: the same corners are read), which the batch keeps when they
// win.  The choice is stored per size class (storage type, transfer function, smoothing,
// and the log2 buckets of the batch size, the median voxel count and the median image
// size) in a text cache file that later batches of the same class reuse without timing.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "march.h"

namespace svr {

struct BatchVol {
    VolDesc v;
    svr_camera cam;
    float4* out;
    int32_t tiles_x;
};

struct BatchArgs {
    const BatchVol* vols;
    const int2* items;     // (volume, tile)
    int32_t nitems;
    int32_t* counter;
    const float4* lut;
    int32_t lut_n;
    svr_params p;
    int32_t tw;            // waves per tile along x (1, 2 or 4); tile = 8*tw x 8*(4/tw)
};

__global__ void batch_reset_kernel(int32_t* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0;
}

// Fetch slots of the batched sample loop: the persistent kernel keeps fewer registers free
// than the one-cube kernel, and AVIP is fastest here with two samples in flight, MIP with
// five (measured on the 512 FP16 sub-cubes).  The batched loop converts 16-bit corners as
// they arrive: keeping them packed (as the one-cube kernel does) measured 2% slower here.
template <int MODE>
constexpr int batch_slots() {
    return (MODE == SVR_MIP0 || MODE == SVR_MIP1 || MODE == SVR_MIPRGB) ? 6 : 3;
}

template <int MODE, int DT, int C, bool WIDE>
__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchArgs b) {
    extern __shared__ float4 smem[];
    __shared__ int s_item;
    float4* s_lut = smem;
    const int n_lut = b.lut_n;
    stage_table(s_lut, b.lut, n_lut);
    float* ring = reinterpret_cast<float*>(smem + n_lut + 1) + threadIdx.x;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int tw = b.tw, th = 4 / tw;
    const int wx = w % tw, wy = w / tw;
    for (;;) {
        __syncthreads();  // the previous item is finished and s_item may be rewritten
        if (threadIdx.x == 0) s_item = atomicAdd(b.counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= b.nitems) break;  // uniform across the workgroup
        const int2 item = b.items[it];
        const BatchVol& bv = b.vols[item.x];
        const int tx = item.y % bv.tiles_x, ty = item.y / bv.tiles_x;
        int lx, ly;
        wave_pixel<DT>(l, lx, ly);
        const int px = tx * (8 * tw) + wx * 8 + lx;
        const int py = ty * (8 * th) + wy * 8 + ly;
        const bool inside = px < bv.cam.width && py < bv.cam.height;
        {
            RenderArgs a;
            a.v = bv.v;
            a.v2 = bv.v;
            a.cam = bv.cam;
            a.lut = b.lut;
            a.lut_n = n_lut;
            a.p = b.p;
            a.out = bv.out;
            a.samples = nullptr;
            a.tiles_x = 0;
            a.nblocks = 0;
            float4 res;
            int count;
            render_ray<MODE, 0, DT, C, WIDE, DT == SVR_F32, kSmoothAuto, batch_slots<MODE>(), false>(
                a, s_lut, ring, px, py, inside, res, count);
            if (inside) bv.out[(size_t)py * bv.cam.width + px] = res;
        }
    }
}

using BatchFn = void (*)(BatchArgs);

template <int DT, int C, bool WIDE>
static BatchFn batch_pick(int mode) {
    switch (mode) {
        case SVR_MIP0: return batch_kernel<SVR_MIP0, DT, C, WIDE>;
        case SVR_MIP1: return batch_kernel<SVR_MIP1, DT, C, WIDE>;
        case SVR_MIPRGB: return batch_kernel<SVR_MIPRGB, DT, C, WIDE>;
        case SVR_AVIP0: return batch_kernel<SVR_AVIP0, DT, C, WIDE>;
        case SVR_AVIP1: return batch_kernel<SVR_AVIP1, DT, C, WIDE>;
        default: return batch_kernel<SVR_AVIPRGB, DT, C, WIDE>;
    }
}

template <bool WIDE>
static BatchFn batch_pick_dt(int dtype, int brick, int mode) {
    if (brick == 16) {
        if (dtype == SVR_F16) return batch_pick<SVR_F16, 16, WIDE>(mode);
        if (dtype == SVR_BF16) return batch_pick<SVR_BF16, 16, WIDE>(mode);
        return batch_pick<SVR_F32, 16, WIDE>(mode);
    }
    if (dtype == SVR_F16) return batch_pick<SVR_F16, 8, WIDE>(mode);
    if (dtype == SVR_BF16) return batch_pick<SVR_BF16, 8, WIDE>(mode);
    return batch_pick<SVR_F32, 8, WIDE>(mode);
}

static BatchFn batch_pick_any(int dtype, int brick, bool wide, int mode) {
    return wide ? batch_pick_dt<true>(dtype, brick, mode)
                : batch_pick_dt<false>(dtype, brick, mode);
}

// Host estimate of the samples a tile costs: the longest chord among its four corner rays
// and its centre ray, in steps of dt (0 when all five miss).
static double tile_cost(const svr_camera& c, const VolDesc& v, int x0, int y0, int w, int h,
                        double dt) {
    const int xs[5] = {x0, std::min(x0 + w - 1, c.width - 1), x0,
                       std::min(x0 + w - 1, c.width - 1), std::min(x0 + w / 2, c.width - 1)};
    const int ys[5] = {y0, y0, std::min(y0 + h - 1, c.height - 1),
                       std::min(y0 + h - 1, c.height - 1), std::min(y0 + h / 2, c.height - 1)};
    double best = 0.0;
    for (int i = 0; i < 5; ++i) {
        const double u = 2.0 * (xs[i] + 0.5) / c.width - 1.0;
        const double vv = 2.0 * (ys[i] + 0.5) / c.height - 1.0;
        double o[3], d[3];
        for (int a = 0; a < 3; ++a) {
            if (c.type == 0) {
                o[a] = c.eye[a] + u * c.U[a] + vv * c.V[a];
                d[a] = c.W[a];
            } else {
                o[a] = c.eye[a];
                d[a] = c.W[a] + u * c.U[a] + vv * c.V[a];
            }
        }
        const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const int n[3] = {v.nx, v.ny, v.nz};
        double tn = 0.0, tf = INFINITY;
        bool hit = len > 0.0;
        for (int a = 0; a < 3 && hit; ++a) {
            const double da = d[a] / len;
            if (da == 0.0) {
                hit = o[a] >= -0.5 && o[a] <= n[a] - 0.5;
                continue;
            }
            double ta = (-0.5 - o[a]) / da, tb = (n[a] - 0.5 - o[a]) / da;
            if (ta > tb) std::swap(ta, tb);
            tn = std::max(tn, ta);
            tf = std::min(tf, tb);
        }
        if (hit && tf > tn) best = std::max(best, (tf - tn) / dt);
    }
    return best;
}

svr_status check_camera(const svr_camera* c);
svr_status check_lut(const svr_lut* l);
svr_status check_params(const svr_params* p, const svr_volume* v);

}  // namespace svr

using namespace svr;

struct svr_batch {
    int n = 0;
    int mode = 0, dtype = 0, brick = 8;
    std::vector<svr_volume*> copies;  // re-bricked copies of the volumes (library-owned)
    int from_cache = 0;
    float default_ms = 0.0f, tuned_ms = 0.0f;
    BatchVol* d_vols = nullptr;
    int2* d_items = nullptr;
    size_t items_cap = 0;
    int32_t* d_counter = nullptr;
    BatchArgs args{};
    BatchFn fn = nullptr;
    int grid = 0;
    size_t lds = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<BatchVol> vols;
    svr_lut lut{};
};

static void free_copies(std::vector<svr_volume*>& c) {
    for (svr_volume* v : c) (void)svr_volume_destroy(v);
    c.clear();
}

static void batch_free(svr_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_vols) (void)hipFree(b->d_vols);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_counter) (void)hipFree(b->d_counter);
    free_copies(b->copies);
    delete b;
}

// ---------------------------------------------------------------- tuning cache
// One line per size class: "<key> <brick> <tile_waves_x> <workgroups per CU>".
static std::mutex g_cache_mu;
static std::string g_cache_path;  // empty: no cache file
static bool g_cache_set = false;  // set by svr_set_tune_cache (else SVR_TUNE_CACHE is read)

static void cache_default() {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (g_cache_set) return;
    const char* env = getenv("SVR_TUNE_CACHE");
    g_cache_path = env ? env : "";
    g_cache_set = true;
}

static int log2_bucket(double x) { return x >= 1.0 ? (int)floor(log2(x)) : 0; }

static std::string size_class(const svr_batch* b, const svr_volume* const* vols, int cus) {
    std::vector<double> vox(b->n), pix(b->n);
    for (int i = 0; i < b->n; ++i) {
        vox[i] = (double)vols[i]->d.nx * vols[i]->d.ny * vols[i]->d.nz;
        pix[i] = (double)b->vols[i].cam.width * b->vols[i].cam.height;
    }
    std::nth_element(vox.begin(), vox.begin() + b->n / 2, vox.end());
    std::nth_element(pix.begin(), pix.begin() + b->n / 2, pix.end());
    char key[160];
    snprintf(key, sizeof key, "dtype%d_mode%d_box%d_n%d_vox%d_pix%d_cu%d", b->dtype, b->mode,
             b->args.p.box_arm > 0 ? 1 : 0, log2_bucket(b->n), log2_bucket(vox[b->n / 2]),
             log2_bucket(pix[b->n / 2]), cus);
    return key;
}

static bool cache_lookup(const std::string& key, int* brick, int* tw, int* per_cu) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (g_cache_path.empty()) return false;
    FILE* f = fopen(g_cache_path.c_str(), "r");
    if (!f) return false;
    char k[160];
    int br, t, pc;
    bool found = false;
    while (fscanf(f, "%159s %d %d %d", k, &br, &t, &pc) == 4) {
        if (key == k && (br == 8 || br == 16) && (t == 1 || t == 2 || t == 4) && pc >= 1 &&
            pc <= 64) {  // the last entry for the key wins
            *brick = br;
            *tw = t;
            *per_cu = pc;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const std::string& key, int brick, int tw, int per_cu) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (g_cache_path.empty()) return;
    FILE* f = fopen(g_cache_path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d\n", key.c_str(), brick, tw, per_cu);
    fclose(f);
}

// Copies of the batch's volumes with brick edge `brick`: each exported to a linear cube of
// its storage type and uploaded again (an exact copy, same values and min/max).
static svr_status rebrick(const svr_volume* const* vols, int n, int brick, hipStream_t s,
                          std::vector<svr_volume*>& out) {
    size_t most = 0;
    for (int i = 0; i < n; ++i)
        most = std::max(most, (size_t)vols[i]->d.nx * vols[i]->d.ny * vols[i]->d.nz *
                                  (vols[i]->d.dtype == SVR_F32 ? 4 : 2));
    void* lin = nullptr;
    svr_status st = hip_fail(hipMalloc(&lin, most), "re-brick buffer");
    for (int i = 0; i < n && !st; ++i) {
        st = svr_volume_export(vols[i], lin, s);
        svr_cube_view cv{lin, vols[i]->d.dtype, vols[i]->d.nx, vols[i]->d.ny, vols[i]->d.nz,
                         0, 0, 0};
        svr_volume* v = nullptr;
        if (!st) st = svr_volume_create(&cv, vols[i]->d.dtype, brick, NAN, s, &v);
        if (!st) out.push_back(v);
    }
    if (lin) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(lin);
    }
    if (st) free_copies(out);
    return st;
}

// Build the cost-ordered queue for tile shape tw and upload it.
static svr_status batch_items(svr_batch* b, int tw, hipStream_t s) {
    const int th = 4 / tw, tile_w = 8 * tw, tile_h = 8 * th;
    std::vector<std::pair<double, int2>> q;
    for (int i = 0; i < b->n; ++i) {
        BatchVol& bv = b->vols[i];
        bv.tiles_x = (bv.cam.width + tile_w - 1) / tile_w;
        const int tiles_y = (bv.cam.height + tile_h - 1) / tile_h;
        for (int t = 0; t < bv.tiles_x * tiles_y; ++t) {
            const int x0 = (t % bv.tiles_x) * tile_w, y0 = (t / bv.tiles_x) * tile_h;
            q.push_back({tile_cost(bv.cam, bv.v, x0, y0, tile_w, tile_h, b->args.p.dt),
                         make_int2(i, t)});
        }
    }
    std::stable_sort(q.begin(), q.end(),
                     [](const std::pair<double, int2>& x, const std::pair<double, int2>& y) {
                         return x.first > y.first;
                     });
    std::vector<int2> items(q.size());
    for (size_t i = 0; i < q.size(); ++i) items[i] = q[i].second;
    // the queue length depends on the tile shape: (re)allocate when this one is longer
    if (items.size() > b->items_cap) {
        if (b->d_items) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(b->d_items);
            b->d_items = nullptr;
            b->items_cap = 0;
        }
        hipError_t e = hipMalloc(&b->d_items, items.size() * sizeof(int2));
        if (e != hipSuccess) return hip_fail(e, "batch queue allocation");
        b->items_cap = items.size();
    }
    if (b->d_vols == nullptr) {
        hipError_t e = hipMalloc(&b->d_vols, b->vols.size() * sizeof(BatchVol));
        if (e != hipSuccess) return hip_fail(e, "batch descriptor allocation");
    }
    svr_status st = hip_fail(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(int2),
                                            hipMemcpyHostToDevice, s), "batch queue upload");
    if (st) return st;
    st = hip_fail(hipMemcpyAsync(b->d_vols, b->vols.data(), b->vols.size() * sizeof(BatchVol),
                                 hipMemcpyHostToDevice, s), "batch descriptor upload");
    if (st) return st;
    // the host vectors are released on return: finish the copies first
    st = hip_fail(hipStreamSynchronize(s), "batch upload sync");
    b->args.items = b->d_items;
    b->args.vols = b->d_vols;
    b->args.nitems = (int32_t)items.size();
    b->args.tw = tw;
    return st;
}

static svr_status batch_enqueue(const svr_batch* b, int grid, hipStream_t s);

// Median of three timed launches of the current queue at `grid` workgroups, after a warm-up.
static svr_status batch_time(const svr_batch* b, int grid, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1, float* median_ms) {
    svr_status st = batch_enqueue(b, grid, s);
    float ms[3] = {0.0f, 0.0f, 0.0f};
    for (int r = 0; r < 3 && !st; ++r) {
        st = hip_fail(hipEventRecord(e0, s), "autotune event");
        if (!st) st = batch_enqueue(b, grid, s);
        if (!st) st = hip_fail(hipEventRecord(e1, s), "autotune event");
        if (!st) st = hip_fail(hipEventSynchronize(e1), "autotune");
        if (!st) st = hip_fail(hipEventElapsedTime(&ms[r], e0, e1), "autotune time");
    }
    std::sort(ms, ms + 3);
    *median_ms = ms[1];
    return st;
}

static svr_status batch_enqueue(const svr_batch* b, int grid, hipStream_t s) {
    // every table the persistent kernel reads must be in place and sized for the queue
    if (!b->args.items || !b->args.vols || !b->args.counter || !b->args.lut ||
        (size_t)b->args.nitems > b->items_cap || b->args.nitems < 1 ||
        !(b->args.tw == 1 || b->args.tw == 2 || b->args.tw == 4) || grid < 1) {
        set_error("batch: internal queue not ready");
        return SVR_EINVAL;
    }
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, b->d_counter);
    hipLaunchKernelGGL(b->fn, dim3(grid), dim3(kBlock), b->lds, s, b->args);
    return hip_fail(hipGetLastError(), "batch launch");
}

extern "C" {

svr_status svr_batch_create(const svr_volume* const* vols, const svr_camera* cams, int32_t n,
                            const svr_lut* lut, const svr_params* params,
                            float* const* rgba_outs, int32_t tune, void* stream,
                            svr_batch** out) {
    if (!vols || !cams || !rgba_outs || !out || n < 1) {
        set_error("svr_batch_create: null argument or n < 1");
        return SVR_EINVAL;
    }
    if (tune < 0 || tune > 2) {
        set_error("svr_batch_create: tune = %d (0, 1 or 2)", tune);
        return SVR_EINVAL;
    }
    cache_default();
    svr_status st = check_lut(lut);
    if (st) return st;
    if ((st = check_params(params, vols[0]))) return st;
    if (params->star_n != 0) {
        set_error("svr_batch_create: the in-ray Gaussian (star_n > 0) is not available in "
                  "batched launches");
        return SVR_EINVAL;
    }
    if (params->ratio != 0) {
        set_error("svr_batch_create: line-ratio methods are not batched");
        return SVR_EINVAL;
    }
    for (int i = 0; i < n; ++i) {
        if (!vols[i] || !rgba_outs[i]) {
            set_error("svr_batch_create: null volume or output %d", i);
            return SVR_EINVAL;
        }
        if (!aligned_to(rgba_outs[i], 16)) {
            set_error("svr_batch_create: output %d not 16-byte aligned", i);
            return SVR_EINVAL;
        }
        if ((st = check_camera(&cams[i]))) return st;
        if ((st = check_params(params, vols[i]))) return st;
        if (vols[i]->d.dtype != vols[0]->d.dtype || vols[i]->d.brick != vols[0]->d.brick) {
            set_error("svr_batch_create: all volumes must share storage type and brick size");
            return SVR_EINVAL;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    svr_batch* b = new (std::nothrow) svr_batch;
    if (!b) return SVR_ENOMEM;
    b->n = n;
    b->mode = params->mode;
    b->dtype = vols[0]->d.dtype;
    b->brick = vols[0]->d.brick;
    b->lut = *lut;
    b->vols.resize(n);
    for (int i = 0; i < n; ++i) {
        b->vols[i].v = vols[i]->d;
        b->vols[i].cam = cams[i];
        b->vols[i].out = reinterpret_cast<float4*>(rgba_outs[i]);
    }
    b->args.lut = reinterpret_cast<const float4*>(lut->rgba);
    b->args.lut_n = lut->n;
    b->args.p = *params;
    b->lds = render_lds_bytes(lut->n, params->box_arm, 0);
    hipError_t e = hipMalloc(&b->d_counter, 64);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "batch counter allocation");
    }
    b->args.counter = b->d_counter;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);

    // default shape: the caller's brick edge, 16 x 16 pixel tiles, 4 workgroups per CU
    const int native = b->brick, other = native == 8 ? 16 : 8;
    int best_brick = native, best_tw = 2, best_pc = 4;
    std::vector<svr_volume*>& copies = b->copies;
    auto use_brick = [&](int brick) -> svr_status {
        bool wide = false;
        for (int i = 0; i < n; ++i) {
            const svr_volume* v = brick == native ? vols[i] : copies[i];
            b->vols[i].v = v->d;
            wide = wide || wide_volume(v->d);
        }
        b->fn = batch_pick_any(b->dtype, brick, wide, b->mode);
        return SVR_OK;
    };
    if (tune) {
        const std::string key = size_class(b, vols, cus);
        int cb = 0, ct = 0, cp = 0;
        if (tune == 1 && cache_lookup(key, &cb, &ct, &cp)) {
            best_brick = cb;
            best_tw = ct;
            best_pc = cp;
            b->from_cache = 1;
        } else {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            st = hip_fail(hipEventCreate(&e0), "autotune event");
            if (!st) st = hip_fail(hipEventCreate(&e1), "autotune event");
            float best_ms = INFINITY;
            const int bricks[2] = {native, other};
            const int tws[3] = {2, 4, 1};
            const int per_cu[3] = {4, 8, 2};
            for (int bi = 0; bi < 2 && !st; ++bi) {
                if (bricks[bi] != native && copies.empty())
                    st = rebrick(vols, n, bricks[bi], s, copies);
                if (!st) st = use_brick(bricks[bi]);
                for (int ti = 0; ti < 3 && !st; ++ti) {
                    st = batch_items(b, tws[ti], s);
                    for (int gi = 0; gi < 3 && !st; ++gi) {
                        float ms = 0.0f;
                        st = batch_time(b, cus * per_cu[gi], s, e0, e1, &ms);
                        if (st) break;
                        if (bi == 0 && ti == 0 && gi == 0) b->default_ms = ms;
                        if (ms < best_ms) {
                            best_ms = ms;
                            best_brick = bricks[bi];
                            best_tw = tws[ti];
                            best_pc = per_cu[gi];
                        }
                    }
                }
            }
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (!st) {
                b->tuned_ms = best_ms;
                cache_store(key, best_brick, best_tw, best_pc);
            }
        }
    }
    // keep re-bricked copies only when their brick edge was chosen
    if (!st && best_brick == native) free_copies(copies);
    if (!st && best_brick != native && copies.empty())
        st = rebrick(vols, n, best_brick, s, copies);
    if (!st) st = use_brick(best_brick);
    b->brick = best_brick;
    const int best_grid = cus * best_pc;
    if (!st) st = batch_items(b, best_tw, s);
    b->grid = best_grid;
    if (!st) {
        hipStream_t cap = nullptr;
        st = hip_fail(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
        if (!st) {
            st = hip_fail(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal),
                          "begin capture");
            if (!st) {
                const svr_status sq = batch_enqueue(b, b->grid, cap);
                st = hip_fail(hipStreamEndCapture(cap, &b->graph), "end capture");
                if (sq) st = sq;
            }
            if (!st)
                st = hip_fail(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0),
                              "graph instantiate");
            (void)hipStreamDestroy(cap);
        }
    }
    if (st) {
        batch_free(b);
        return st;
    }
    *out = b;
    return SVR_OK;
}

svr_status svr_batch_launch(svr_batch* batch, void* stream) {
    if (!batch) {
        set_error("svr_batch_launch: null batch");
        return SVR_EINVAL;
    }
    return hip_fail(hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream)),
                    "batch graph launch");
}

svr_status svr_batch_info(const svr_batch* batch, svr_batch_stats* stats) {
    if (!batch || !stats) {
        set_error("svr_batch_info: null argument");
        return SVR_EINVAL;
    }
    stats->items = batch->args.nitems;
    stats->grid = batch->grid;
    stats->tile_waves_x = batch->args.tw;
    stats->brick = batch->brick;
    stats->from_cache = batch->from_cache;
    stats->default_ms = batch->default_ms;
    stats->tuned_ms = batch->tuned_ms;
    return SVR_OK;
}

svr_status svr_set_tune_cache(const char* path) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache_path = path ? path : "";
    g_cache_set = true;
    return SVR_OK;
}

svr_status svr_batch_destroy(svr_batch* batch) {
    if (batch) (void)hipDeviceSynchronize();
    batch_free(batch);
    return SVR_OK;
}

}  // extern "C"
