// Host-side exhaustive check of the bricked addressing the ray-march and the export use
// (tests/test_sanitizers.py builds it with AddressSanitizer and UndefinedBehaviorSanitizer
// on the host code): for ragged volumes of every storage type at brick edges 8 and 16,
//  - every cell a trilinear fetch can select (each coordinate in [0, n-1]) reads elements
//    [cell_offset, cell_offset + corner_span] inside the storage (bricks x pitch);
//  - every voxel's stored element (brick_loc) lies inside its brick's pitch, and no two
//    voxels share one (float32), or pair slot (16-bit y-pairs: voxel y sits in the pair of
//    y and, as the second half, in the pair of y - 1 within a brick).
// Also the workgroup -> tile maps of the grids (xcd_tile, xcd_run_tile): each is a bijection
// of [0, nblocks) that keeps a workgroup on the XCD it is dispatched to (b mod 8), for every
// grid size up to 20,000 tiles, and xcd_run_tile gives every XCD one run in each aligned
// window of eight runs.
// Exit status 0 when every check holds; a message and status 1 otherwise.
#include <stdio.h>

#include <vector>

#include "common.h"

using namespace svr;

template <int DT, int C>
static int check(int nx, int ny, int nz) {
    const VolDesc d = make_voldesc(nx, ny, nz, DT, C);
    const uint64_t storage = (uint64_t)d.nbx * d.nby * d.nbz * d.pitch;
    if (storage >= (1ull << 32)) return 0;  // such volumes use 64-bit addressing
    if ((uint64_t)brick_elems(DT, C) > d.pitch) {
        printf("pitch %u below brick elements %d\n", d.pitch, brick_elems(DT, C));
        return 1;
    }
    std::vector<unsigned char> seen(storage, 0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const uint64_t o = cell_offset<DT, C>(x, y, z, d.nbx, d.nby, d.pitch);
                if (o + corner_span<DT, C>() >= storage) {
                    printf("DT %d C %d dims %d %d %d: cell (%d %d %d) reads up to %llu of %llu\n",
                           DT, C, nx, ny, nz, x, y, z,
                           (unsigned long long)(o + corner_span<DT, C>()),
                           (unsigned long long)storage);
                    return 1;
                }
                const uint64_t b = ((uint64_t)(z / C) * d.nby + y / C) * d.nbx + x / C;
                const uint32_t loc = brick_loc<DT, C>(x % C, y % C, z % C);
                if (o != b * d.pitch + loc || loc + (DT == SVR_F32 ? 0u : 1u) >= d.pitch) {
                    printf("DT %d C %d: voxel (%d %d %d) at %llu, brick %llu loc %u\n", DT, C, x,
                           y, z, (unsigned long long)o, (unsigned long long)b, loc);
                    return 1;
                }
                if (seen[o]++) {
                    printf("DT %d C %d: voxel (%d %d %d) shares element %llu\n", DT, C, x, y, z,
                           (unsigned long long)o);
                    return 1;
                }
            }
    return 0;
}

// The tile maps over a grid of n workgroups (see the file comment).
static int check_tile_maps(int n) {
    std::vector<int> owner(n), a(n, -1), b(n, -1);
    for (int i = 0; i < n; ++i) {
        const int t = xcd_tile(i, n), u = xcd_run_tile(i, n);
        if (t < 0 || t >= n || a[t] >= 0 || u < 0 || u >= n || b[u] >= 0) {
            printf("tile maps over %d workgroups: workgroup %d -> %d / %d is not a bijection\n",
                   n, i, t, u);
            return 1;
        }
        a[t] = i;
        b[u] = i;
    }
    // xcd_run_tile: each aligned window of 8 runs holds one run of every XCD
    const int win = 8 * kXcdRun;
    for (int w0 = 0; w0 + win <= n; w0 += win) {
        int cnt[8] = {0};
        for (int t = w0; t < w0 + win; ++t) cnt[b[t] & 7]++;
        for (int x = 0; x < 8; ++x)
            if (cnt[x] != kXcdRun) {
                printf("tile maps over %d workgroups: XCD %d owns %d tiles of [%d, %d)\n", n, x,
                       cnt[x], w0, w0 + win);
                return 1;
            }
    }
    return 0;
}

int main() {
    int maps_bad = 0;
    for (int n = 1; n <= 20000; ++n) maps_bad |= check_tile_maps(n);
    printf("tile maps: grids of 1..20000 workgroups %s\n", maps_bad ? "FAILED" : "ok");

    const int dims[][3] = {{1, 1, 1}, {2, 1, 1}, {7, 9, 13}, {8, 8, 8}, {9, 17, 33},
                           {16, 16, 16}, {17, 1, 2}, {100, 3, 65}, {45, 37, 70}, {64, 64, 64},
                           {33, 130, 5}};
    int bad = 0, n = 0;
    for (const auto& v : dims) {
        bad |= check<SVR_F32, 8>(v[0], v[1], v[2]);
        bad |= check<SVR_F32, 16>(v[0], v[1], v[2]);
        bad |= check<SVR_F16, 8>(v[0], v[1], v[2]);
        bad |= check<SVR_F16, 16>(v[0], v[1], v[2]);
        bad |= check<SVR_BF16, 8>(v[0], v[1], v[2]);
        bad |= check<SVR_BF16, 16>(v[0], v[1], v[2]);
        n += 6;
    }
    printf("brick addressing: %d volume layouts checked, %s\n", n, bad ? "FAILED" : "ok");
    return bad | maps_bad;
}
