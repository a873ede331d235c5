// Tile binning: per-tile, depth-ordered splat lists.
//
// The ordering key of an instance is (global tile id, FP32 depth bits,
// entry id).  It is built as an LSD radix sort whose depth digits are applied
// per entry rather than per instance (every instance of an entry shares its
// depth, so sorting the entries by depth and emitting their instances in that
// order is exactly the result of the depth passes), followed by stable
// passes on the tile id alone.  That moves 8 bytes per instance per tile
// pass instead of 12 bytes per instance for each of ~6 passes over 64-bit
// keys.
//
//   flags = tiles_touched > 0  -> exclusive scan -> compact visible entries
//   radix sort (depth bits, entry) over the visible entries
//   gather tiles_touched in depth order -> exclusive scan -> instance offsets
//   emit (tile, entry) for every tile of each footprint rectangle, row-major
//   radix sort on the tile id (stable)
//   tile ranges from adjacent keys;  optional heavy-first tile order
#include "gs_internal.h"

namespace {

__global__ void flag_visible_kernel(const u32* tiles_touched, u32* flags, int64_t E) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < E) flags[i] = tiles_touched[i] > 0 ? 1u : 0u;
}

__global__ void compact_kernel(const u32* tiles_touched, const u32* offs, const u32* depth_key,
                               u32* keys, u32* vals, int64_t E) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E || tiles_touched[e] == 0) return;
    const u32 j = offs[e];
    keys[j] = depth_key[e];
    vals[j] = (u32)e;
}

__global__ void gather_counts_kernel(const u32* vals, const u32* tiles_touched, u32* cnt,
                                     const u32* n_vis, int64_t E) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= E || j >= (int64_t)*n_vis) return;
    const u32 e = vals[j];
    cnt[j] = e < (u64)E ? tiles_touched[e] : 0u;
}

// counters[5] = min(instances, capacity): the length the tile sort works on
__global__ void clamp_count_kernel(u32* counters, u32 cap) {
    const u32 n = counters[1];
    counters[5] = n < cap ? n : cap;
    counters[2] = n > cap ? 1u : 0u;
}

__global__ void emit_kernel(const u32* vals, const u32* offs, const uint2* rect,
                            const gs_view_info* views, int64_t n, const u32* n_vis, u32 cap,
                            u32* tile_keys, u32* entries, int64_t E) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= E || j >= (int64_t)*n_vis) return;
    const u32 e = vals[j];
    if (e >= (u64)E) return;
    const int v = (int)(e / (u64)n);
    const gs_view_info vi = views[v];
    const uint2 r = rect[e];
    const u32 x0 = r.x & 0xffffu, x1 = r.x >> 16, y0 = r.y & 0xffffu, y1 = r.y >> 16;
    u32 o = offs[j];
    for (u32 ty = y0; ty <= y1; ++ty) {
        const u32 row = (u32)vi.tile_base + ty * (u32)vi.tiles_x;
        for (u32 tx = x0; tx <= x1; ++tx) {
            if (o < cap) {
                tile_keys[o] = row + tx;
                entries[o] = e;
            }
            ++o;
        }
    }
}

__global__ void ranges_kernel(const u32* keys, const u32* n_ptr, uint2* ranges, u32 T) {
    const u32 n = *n_ptr;
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 k = keys[i];
    if (k >= T) return;
    if (i == 0 || keys[i - 1] != k) ranges[k].x = i;
    if (i == n - 1 || keys[i + 1] != k) ranges[k].y = i + 1;
}

// heavy-first order key: longer lists first, ties by tile id (stable sort)
__global__ void tile_weight_kernel(const uint2* ranges, u32* keys, u32* vals, int T) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    u32 len = ranges[t].y - ranges[t].x;
    if (len > 0xFFFFFFu) len = 0xFFFFFFu;
    keys[t] = 0xFFFFFFu - len;
    vals[t] = (u32)t;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + GS_BLOCK - 1) / GS_BLOCK); }

}  // namespace

gs_status gs_launch_bin(gs_frame* f, hipStream_t s, bool heavy_first) {
    const int64_t E = f->E;
    u32* cnt = f->counters;
    if (E > 0) {
        flag_visible_kernel<<<blocks_for(E), GS_BLOCK, 0, s>>>(f->tiles_touched, f->flags, E);
        GS_TRY(gs_check_launch("flag_visible"));
        GS_TRY(gs_scan_exclusive(f->flags, f->flags, nullptr, (u32)E, cnt + 0, f->scan_part, s));
        compact_kernel<<<blocks_for(E), GS_BLOCK, 0, s>>>(f->tiles_touched, f->flags, f->depth_key,
                                                          f->vkeys[0], f->vvals[0], E);
        GS_TRY(gs_check_launch("compact"));
        // depths are positive, so the sign bit is zero: 31 key bits
        GS_TRY(gs_radix_sort(f->vkeys, f->vvals, cnt + 0, 0, 31, f->G_vis, f->radix_hist,
                             f->scan_part, &f->vsorted, s));
        const u32* sv = f->vvals[f->vsorted];
        gather_counts_kernel<<<blocks_for(E), GS_BLOCK, 0, s>>>(sv, f->tiles_touched, f->inst_off,
                                                                cnt + 0, E);
        GS_TRY(gs_check_launch("gather_counts"));
        GS_TRY(gs_scan_exclusive(f->inst_off, f->inst_off, cnt + 0, 0, cnt + 1, f->scan_part, s));
        clamp_count_kernel<<<1, 1, 0, s>>>(cnt, (u32)f->cap);
        GS_TRY(gs_check_launch("clamp_count"));
        emit_kernel<<<blocks_for(E), GS_BLOCK, 0, s>>>(sv, f->inst_off, f->rect, f->d_views, f->n,
                                                       cnt + 0, (u32)f->cap, f->ikeys[0],
                                                       f->ivals[0], E);
        GS_TRY(gs_check_launch("emit"));
        GS_TRY(gs_radix_sort(f->ikeys, f->ivals, cnt + 5, 0, f->tile_bits, f->G_inst,
                             f->radix_hist, f->scan_part, &f->isorted, s));
    } else {
        GS_TRY(gs_fill_u32(cnt, 0u, 8, s));
    }
    GS_TRY(gs_fill_u32((u32*)f->ranges, 0u, 2 * (int64_t)f->T, s));
    ranges_kernel<<<blocks_for(f->cap), GS_BLOCK, 0, s>>>(f->ikeys[f->isorted], cnt + 5, f->ranges,
                                                              (u32)f->T);
    GS_TRY(gs_check_launch("ranges"));
    if (heavy_first) {
        tile_weight_kernel<<<blocks_for(f->T), GS_BLOCK, 0, s>>>(f->ranges, f->tkeys[0], f->tvals[0],
                                                                 f->T);
        GS_TRY(gs_check_launch("tile_weight"));
        GS_TRY(gs_radix_sort(f->tkeys, f->tvals, nullptr, (u32)f->T, 24, f->G_tile, f->radix_hist,
                             f->scan_part, &f->tsorted, s));
    }
    return GS_OK;
}
