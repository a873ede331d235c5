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

// Scan epilogue of the visibility flags: entry i with flag 1 goes to slot
// ex of the compacted (depth key, entry) arrays; the total is the number of
// visible entries.
struct CompactEpi {
    const u32* depth_key;
    u32* keys;
    u32* vals;
    u32* n_visible;
    __device__ void item(u32 i, u32 flag, u32 ex) const {
        if (flag) {
            keys[ex] = depth_key[i];
            vals[ex] = i;
        }
    }
    __device__ void finish(u32 t) const { *n_visible = t; }
};

// Instance emission, balanced per 256 instances.  Pass 1 records, for every
// chunk of 256 consecutive instance slots, the depth-sorted entry whose tiles
// start the chunk.  Pass 2 gives each workgroup whole chunks: it stages the
// (at most 256) entries a chunk can touch in LDS, and each thread finds the
// entry of its slot by binary search over their offsets (strictly
// increasing: every visible entry has at least one tile), then writes
// (tile, entry) for the k-th tile of the rectangle, row-major.  Depth order
// puts the largest footprints (nearest Gaussians) together, so balancing on
// instances rather than on entries is what keeps the workgroups even.
constexpr u32 EMIT_CHUNK = 256;

// Scan epilogue of the tile counts in depth order: the instance offset of
// visible entry j, and for every chunk of 256 instance slots that starts
// inside its range the entry j itself (chunk_start, below the capacity); the
// last workgroup publishes the instance total, the kept length min(total,
// capacity) the tile sort works on, and the overflow flag.
struct ChunkEpi {
    u32* inst_off;
    u32* chunk_start;
    u32* counters;
    u32 cap;
    __device__ void item(u32 j, u32 tt, u32 off) const {
        inst_off[j] = off;
        const u64 hi = (u64)off + tt < cap ? (u64)off + tt : cap;
        for (u64 c = ((u64)off + EMIT_CHUNK - 1) / EMIT_CHUNK; c * EMIT_CHUNK < hi; ++c)
            chunk_start[c] = j;
    }
    __device__ void finish(u32 t) const {
        counters[1] = t;
        counters[5] = t < cap ? t : cap;
        counters[2] = t > cap ? 1u : 0u;
    }
};

__global__ void __launch_bounds__(GS_BLOCK) emit_kernel(const u32* vals, const u32* offs,
                                                        const uint2* rect, const float4* splat,
                                                        const gs_view_info* views, int64_t n,
                                                        const u32* n_vis, const u32* n_kept,
                                                        const u32* chunk_start, u32* tile_keys,
                                                        u32* entries, int64_t E, u32 T) {
    __shared__ u32 s_off[EMIT_CHUNK], s_e[EMIT_CHUNK], s_rx[EMIT_CHUNK], s_ry[EMIT_CHUNK];
    __shared__ u32 s_tb[EMIT_CHUNK], s_tw[EMIT_CHUNK];
    __shared__ float4 s_p0[EMIT_CHUNK], s_p1[EMIT_CHUNK];
    const int t = threadIdx.x;
    const u32 nv = *n_vis, kept = *n_kept;
    const u32 chunks = (kept + EMIT_CHUNK - 1) / EMIT_CHUNK;
    for (u32 c = blockIdx.x; c < chunks; c += gridDim.x) {
        // the entries that own instances of this chunk: from its first owner to
        // the owner of the next chunk's first instance
        const u32 j0 = chunk_start[c];
        const u32 j1 = c + 1 < chunks ? chunk_start[c + 1] : nv - 1;
        const u32 span = j1 - j0 + 1;
        const int m = span < EMIT_CHUNK ? (int)span : (int)EMIT_CHUNK;
        __syncthreads();
        if (t < m) {
            u32 e = vals[j0 + t];
            if (e >= (u64)E) e = 0;
            const uint2 r = rect[e];
            int v = 0;
            while ((u64)(v + 1) * (u64)n <= (u64)e) ++v;   // view of the entry (V <= 32)
            s_off[t] = offs[j0 + t];
            s_e[t] = e;
            s_rx[t] = r.x;
            s_ry[t] = r.y;
            s_tb[t] = (u32)views[v].tile_base;
            s_tw[t] = (u32)views[v].tiles_x;
            s_p0[t] = splat[3 * (u64)e];
            s_p1[t] = splat[3 * (u64)e + 1];
        }
        __syncthreads();
        const u32 o = c * EMIT_CHUNK + (u32)t;
        if (o < kept) {
            int lo = 0, hi = m - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid] <= o) lo = mid;
                else hi = mid - 1;
            }
            // the k-th tile of the entry, rows top to bottom, columns left to right,
            // counted exactly as the projection counted them
            u32 k = o - s_off[lo];
            const u32 rx = s_rx[lo], ry = s_ry[lo];
            const int x0 = (int)(rx & 0xffffu), x1 = (int)(rx >> 16);
            const int y0 = (int)(ry & 0xffffu), y1 = (int)(ry >> 16);
            const FootprintRows fr = footprint_rows(s_p0[lo], s_p1[lo]);
            u32 tile = T;   // not reached: the rows hold exactly the counted tiles
            for (int ty = y0; ty <= y1; ++ty) {
                int first = 0;
                const u32 cnt = footprint_row_count(fr, ty, x0, x1, &first);
                if (k < cnt) {
                    tile = s_tb[lo] + (u32)ty * s_tw[lo] + (u32)first + k;
                    break;
                }
                k -= cnt;
            }
            tile_keys[o] = tile;
            entries[o] = s_e[lo];
        }
    }
}

// Tile ranges [start, end) from the sorted tile keys, empty tiles included
// (as an empty range at the position where they would start), so no clearing
// pass is needed: the thread at each boundary i (a change of key between i-1
// and i, or the two ends) closes the previous tile, writes the tiles strictly
// between the two keys and opens the next.  Keys >= T (never produced) count
// as T.
__global__ void ranges_kernel(const u32* keys, const u32* n_ptr, uint2* ranges, u32 T) {
    const u32 n = *n_ptr;
    const u32 stride = gridDim.x * blockDim.x;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
        const int64_t prev = i == 0 ? -1 : (int64_t)(keys[i - 1] < T ? keys[i - 1] : T);
        const int64_t cur = i == n ? (int64_t)T : (int64_t)(keys[i] < T ? keys[i] : T);
        if (cur == prev) continue;
        if (prev >= 0 && prev < (int64_t)T) ranges[prev].y = i;
        for (int64_t t = prev + 1; t < cur && t < (int64_t)T; ++t) ranges[t] = make_uint2(i, i);
        if (cur < (int64_t)T) ranges[cur].x = i;
    }
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
        // flags[e] = (tiles_touched[e] > 0) and counters[6] = 0 come from the projection;
        // the compaction reads them without modifying them, so rendering the same
        // projection again repeats the same work.
        GS_TRY(gs_scan_reduce(f->flags, nullptr, nullptr, (u32)E, f->scan_part, s));
        const CompactEpi ce{f->depth_key, f->vkeys[0], f->vvals[0], cnt + 0};
        scan_down_kernel<CompactEpi><<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(f->flags, nullptr, nullptr,
                                                                      (u32)E, f->scan_part, ce);
        GS_TRY(gs_check_launch("compact"));
        // depths are positive, so the sign bit is zero: 31 key bits
        GS_TRY(gs_radix_sort(f->vkeys, f->vvals, cnt + 0, 0, E, 31, f->sort_scratch, cnt + 6,
                             &f->vsorted, s));
        const u32* sv = f->vvals[f->vsorted];
        // instance offsets: exclusive scan of tiles_touched in depth order, with chunk starts
        GS_TRY(gs_scan_reduce(f->tiles_touched, sv, cnt + 0, 0, f->scan_part, s));
        const ChunkEpi he{f->inst_off, f->chunk_start, cnt, (u32)f->cap};
        scan_down_kernel<ChunkEpi><<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(f->tiles_touched, sv, cnt + 0,
                                                                    0, f->scan_part, he);
        GS_TRY(gs_check_launch("instance_offsets"));
        emit_kernel<<<2048, GS_BLOCK, 0, s>>>(sv, f->inst_off, f->rect, f->splat, f->d_views, f->n, cnt + 0,
                                              cnt + 5, f->chunk_start, f->ikeys[0], f->ivals[0], E,
                                              (u32)f->T);
        GS_TRY(gs_check_launch("emit"));
        GS_TRY(gs_radix_sort(f->ikeys, f->ivals, cnt + 5, 0, f->cap, f->tile_bits, f->sort_scratch,
                             cnt + 6, &f->isorted, s));
    } else {
        GS_TRY(gs_fill_u32(cnt, 0u, 8, s));
    }
    ranges_kernel<<<4096, GS_BLOCK, 0, s>>>(f->ikeys[f->isorted], cnt + 5, f->ranges, (u32)f->T);
    GS_TRY(gs_check_launch("ranges"));
    if (heavy_first) {
        tile_weight_kernel<<<blocks_for(f->T), GS_BLOCK, 0, s>>>(f->ranges, f->tkeys[0], f->tvals[0],
                                                                 f->T);
        GS_TRY(gs_check_launch("tile_weight"));
        GS_TRY(gs_radix_sort(f->tkeys, f->tvals, nullptr, (u32)f->T, f->T, 24, f->sort_scratch,
                             cnt + 6, &f->tsorted, s));
    }
    return GS_OK;
}
