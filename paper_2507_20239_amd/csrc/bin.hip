// Tile binning: per-tile, depth-ordered splat lists.
//
// The order inside a tile's list is (FP32 depth bits, entry id).  Instances
// are grouped by tile with a radix sort on the tile id alone, and each tile's
// list is then put in depth order by one wave that owns it:
//
//   one exclusive scan of (tiles_touched > 0, tiles_touched) -> compacted
//   visible entries and their instance offsets (entry order)
//   emit (tile, entry) for every tile each footprint meets (or, with the
//   3-sigma footprint, every tile of its rectangle), row-major
//   radix sort on the tile id (its first pass need not be stable: the
//   per-tile sort fixes the order inside each list)
//   tile ranges from adjacent keys;  optional heavy-first tile order
//   per tile: sort the list by (depth bits, entry) in registers (one wave up
//   to 512, the workgroup up to 2048), or for longer lists as register-sorted
//   runs of 2048 merged in global memory
//
// A global sort of the visible entries by depth before emission would give
// the same lists; it takes four radix passes over every visible entry, while
// the per-tile sorts are short, independent and need no pass over the keys'
// full width.
#include "gs_internal.h"

namespace {

// Instance emission, balanced per 256 instances.  Pass 1 records, for every
// chunk of 256 consecutive instance slots, the visible entry whose tiles
// start the chunk.  Pass 2 gives each workgroup whole chunks: it stages the
// (at most 256) entries a chunk can touch in LDS.  With the rectangle test,
// and with the ellipse test when the chunk holds many entries (small
// footprints), each thread finds the entry of its slot by binary search over
// their offsets (strictly increasing: every visible entry has at least one
// tile) and the k-th tile of that entry, walking its rows; when the chunk
// holds few entries (footprints of many rows, whose every instance would walk
// them again) the threads first count the tiles of the entries' rows, one
// row each, and each slot then searches the rows.  Balancing on instances
// rather than on entries keeps the workgroups even when a few footprints
// cover many tiles.
constexpr u32 EMIT_CHUNK = 256;
// Chunks of at most this many entries count their rows in passes.
constexpr int EMIT_PASS_MAX_ENTRIES = 48;

// Visible entries and their instance offsets in one scan: each entry adds
// (1 << 32 | tiles) if it has tiles, so the exclusive prefix holds its slot in
// the compacted list (high half) and its instance offset (low half).  The
// epilogue writes the compacted entry, its offset, and for every chunk of 256
// instance slots that starts inside its range the slot itself (chunk_start,
// below the capacity); the last workgroup publishes the visible count, the
// instance total, the kept length min(total, capacity) and the overflow flag.
// A total of 2^32 instances or more would carry into the high half; the first
// launch also sums the tiles alone (64-bit), and such a step is reported as an
// overflow with nothing kept (no capacity holds it), its slots bounded by the
// entry count.
__device__ __forceinline__ u64 vis_pack(u32 tt) { return tt ? ((u64)1 << 32) | tt : 0ull; }

// The slots of the chunks of 256 instance slots that start inside the range
// [off, off + tt) of a visible entry (below the capacity).
__device__ __forceinline__ void mark_chunks(u32* chunk_start, u32 cap, u32 slot, u32 off, u32 tt) {
    const u64 hi = (u64)off + tt < cap ? (u64)off + tt : cap;
    for (u64 c = ((u64)off + EMIT_CHUNK - 1) / EMIT_CHUNK; c * EMIT_CHUNK < hi; ++c)
        chunk_start[c] = slot;
}

struct VisEpi {
    u32* visible;
    u32* inst_off;
    u32* chunk_start;
    u32* counters;
    u32 cap;
    u32 n;           // entries: bound of the compacted slots
    // depth presort: the compacted entries' depth keys instead of their offsets
    const u32* depth_key;
    u32* dkey;
    __device__ void item(u32 e, u32 tt, u32 slot, u32 off) const {
        if (slot >= n) return;   // only after a carry out of the low half
        visible[slot] = e;
        if (dkey) {
            dkey[slot] = depth_key[e];
            return;
        }
        inst_off[slot] = off;
        mark_chunks(chunk_start, cap, slot, off, tt);
    }
    __device__ void finish(u32 nv, u32 t, u64 tiles) const {
        if (tiles >> 32) {
            counters[0] = nv < n ? nv : n;
            counters[1] = 0xffffffffu;
            counters[5] = 0;
            counters[2] = 1;
            counters[6] = 1;
            return;
        }
        counters[0] = nv;
        counters[1] = t;
        counters[5] = t < cap ? t : cap;
        counters[2] = t > cap ? 1u : 0u;
        if (t > cap) counters[6] = 1;   // sticky: cleared only by the caller
    }
};

// part[0 .. GS_SCAN_PARTS): packed partition sums; part[GS_SCAN_PARTS ..
// 2 GS_SCAN_PARTS): tile sums alone
__global__ void __launch_bounds__(GS_BLOCK) vis_reduce_kernel(const u32* tt, u32 n, u64* part) {
    __shared__ u64 lds4[4];
    u32 beg, end;
    chunk_of(n, GS_SCAN_PARTS, blockIdx.x, beg, end);
    u64 s = 0, st = 0;
    u32 i = beg + threadIdx.x;
    // four loads in flight per thread: a partition holds E / 1024 entries
    for (; i + 3 * GS_BLOCK < end; i += 4 * GS_BLOCK) {
        u32 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = tt[i + j * GS_BLOCK];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s += vis_pack(v[j]);
            st += v[j];
        }
    }
    for (; i < end; i += GS_BLOCK) {
        const u32 v = tt[i];
        s += vis_pack(v);
        st += v;
    }
    u64 total, tiles;
    block_exclusive_scan(s, lds4, total);
    __syncthreads();
    block_exclusive_scan(st, lds4, tiles);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = total;
        part[GS_SCAN_PARTS + blockIdx.x] = tiles;
    }
}

__global__ void __launch_bounds__(GS_BLOCK) vis_down_kernel(const u32* tt, u32 n, const u64* part,
                                                            VisEpi epi) {
    __shared__ u64 lds4[4];
    u64 carry = partition_prefix(part, blockIdx.x);
    u64 before;
    block_exclusive_scan(carry, lds4, before);
    carry = before;
    u32 beg, end;
    chunk_of(n, GS_SCAN_PARTS, blockIdx.x, beg, end);
    for (u32 base = beg; base < end; base += GS_BLOCK * 4) {
        u32 t[4];
        u64 s = 0;
        const u32 i0 = base + threadIdx.x * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) t[j] = load_or_zero(tt, i0 + j, end);
#pragma unroll
        for (int j = 0; j < 4; ++j) s += vis_pack(t[j]);
        u64 total;
        u64 ex = block_exclusive_scan(s, lds4, total) + carry;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (t[j]) epi.item(i0 + j, t[j], (u32)(ex >> 32), (u32)ex);
            ex += vis_pack(t[j]);
        }
        carry += total;
    }
    if (blockIdx.x == gridDim.x - 1) {
        u64 tiles = partition_prefix(part + GS_SCAN_PARTS, GS_SCAN_PARTS);
        u64 all;
        __syncthreads();
        block_exclusive_scan(tiles, lds4, all);
        if (threadIdx.x == 0) epi.finish((u32)(carry >> 32), (u32)carry, all);
    }
}

// The footprint row constants of staged entry j.
__device__ __forceinline__ FootprintRows staged_rows(const float (&s)[9][EMIT_CHUNK], int j) {
    FootprintRows f;
    f.l21 = s[0][j];
    f.l22 = s[1][j];
    f.r2 = s[2][j];
    f.ry = s[3][j];
    f.ds = s[4][j];
    f.il11 = s[5][j];
    f.mx = s[6][j];
    f.hy = s[7][j];
    f.ly = s[8][j];
    return f;
}

template <bool SIGMA3>
__global__ void __launch_bounds__(GS_BLOCK) emit_kernel(const u32* visible, const u32* offs,
                                                        const uint2* rect, const float4* splat,
                                                        const gs_view_info* views, int64_t n,
                                                        const u32* n_vis, const u32* n_kept,
                                                        const u32* chunk_start, u32* tile_keys,
                                                        u32* entries, int64_t E, u32 T) {
    // per staged entry: its instance offset, entry, columns x0 | x1 << 16 and
    // rows y0 | y1 << 16, first tile of its view and the view's tiles per row
    __shared__ u32 s_off[EMIT_CHUNK], s_e[EMIT_CHUNK], s_rx[EMIT_CHUNK], s_ry[EMIT_CHUNK];
    __shared__ u32 s_tb[EMIT_CHUNK], s_tw[EMIT_CHUNK];
    // the footprint row constants of each staged entry, computed once per entry
    __shared__ float s_fr[9][EMIT_CHUNK];
    // row passes: the first row slot of each staged entry; per row slot of a
    // pass its first instance, its first tile and its staged entry
    __shared__ u32 s_rs[EMIT_CHUNK], s_roff[EMIT_CHUNK], s_rtile[EMIT_CHUNK];
    __shared__ unsigned char s_rlo[EMIT_CHUNK];
    __shared__ u32 lds4[4];
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
        // with few entries per chunk (footprints of many tiles) the rows are
        // counted once each, in passes; with many (small footprints) every
        // instance walks its entry's rows itself
        const bool passes = !SIGMA3 && m <= EMIT_PASS_MAX_ENTRIES;
        u32 rows = 0;
        __syncthreads();
        if (t < m) {
            u32 e = visible[j0 + t];
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
            const int y0 = (int)(r.y & 0xffffu), y1 = (int)(r.y >> 16);
            rows = y1 >= y0 ? (u32)(y1 - y0 + 1) : 0u;
            if (!SIGMA3) {
                const FootprintRows fr = footprint_rows(splat[3 * (u64)e], splat[3 * (u64)e + 1]);
                s_fr[0][t] = fr.l21;
                s_fr[1][t] = fr.l22;
                s_fr[2][t] = fr.r2;
                s_fr[3][t] = fr.ry;
                s_fr[4][t] = fr.ds;
                s_fr[5][t] = fr.il11;
                s_fr[6][t] = fr.mx;
                s_fr[7][t] = fr.hy;
                s_fr[8][t] = fr.ly;
            }
        }
        const u32 o = c * EMIT_CHUNK + (u32)t;
        if (!passes) {
            __syncthreads();
            if (o < kept) {
                int lo = 0, hi = m - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= o) lo = mid;
                    else hi = mid - 1;
                }
                // the k-th tile of the entry, rows top to bottom, columns left to
                // right, counted exactly as the projection counted them
                u32 k = o - s_off[lo];
                const u32 rx = s_rx[lo], ry = s_ry[lo];
                const int x0 = (int)(rx & 0xffffu), x1 = (int)(rx >> 16);
                const int y0 = (int)(ry & 0xffffu), y1 = (int)(ry >> 16);
                u32 tile = T;   // not reached: the rows hold exactly the counted tiles
                if (SIGMA3) {
                    // every tile of the rectangle
                    const u32 w = (u32)(x1 - x0 + 1);
                    tile = s_tb[lo] + ((u32)y0 + k / w) * s_tw[lo] + (u32)x0 + k % w;
                } else {
                    const FootprintRows fr = staged_rows(s_fr, lo);
                    for (int ty = y0; ty <= y1; ++ty) {
                        int first = 0;
                        const u32 cnt = footprint_row_count(fr, ty, x0, x1, &first);
                        if (k < cnt) {
                            tile = s_tb[lo] + (u32)ty * s_tw[lo] + (u32)first + k;
                            break;
                        }
                        k -= cnt;
                    }
                }
                tile_keys[o] = tile;
                entries[o] = s_e[lo];
            }
            continue;
        }
        // Row passes: the rows of the staged entries in order, a workgroup's
        // width at a time.  Each thread counts the tiles of one row with the
        // projection's row test, a scan of the counts places the rows'
        // instances (the first staged entry's instances start at its offset,
        // and every entry's rows hold exactly the tiles the projection
        // counted), and each instance of the chunk finds its row by binary
        // search.  Passes stop once they reach the end of the chunk.
        u32 nr;
        const u32 rs = block_exclusive_scan(rows, lds4, nr);
        if (t < m) s_rs[t] = rs;
        const u32 end = min(kept, c * EMIT_CHUNK + EMIT_CHUNK);
        u32 base = s_off[0];   // uniform, like every pass total below
        for (u32 p0 = 0; p0 < nr && base < end; p0 += EMIT_CHUNK) {
            __syncthreads();
            const u32 r = p0 + (u32)t;
            u32 cnt = 0, tile0 = 0;
            int lo = 0;
            if (r < nr) {
                // the staged entry that owns row slot r
                int hi = m - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_rs[mid] <= r) lo = mid;
                    else hi = mid - 1;
                }
                const FootprintRows fr = staged_rows(s_fr, lo);
                const u32 rx = s_rx[lo];
                const int ty = (int)(s_ry[lo] & 0xffffu) + (int)(r - s_rs[lo]);
                int first = 0;
                cnt = footprint_row_count(fr, ty, (int)(rx & 0xffffu), (int)(rx >> 16), &first);
                tile0 = s_tb[lo] + (u32)ty * s_tw[lo] + (u32)first;
            }
            u32 tot;
            // rows past the last hold no tiles and start at the pass's end,
            // after every instance of the pass
            s_roff[t] = base + block_exclusive_scan(cnt, lds4, tot);
            s_rtile[t] = tile0;
            s_rlo[t] = (unsigned char)lo;
            __syncthreads();
            if (o < end && o >= base && o - base < tot) {
                // the last row that starts at or before o: rows without tiles
                // start where the next row does, so this is the row holding o
                int lr = 0, hr = EMIT_CHUNK - 1;
                while (lr < hr) {
                    const int mid = (lr + hr + 1) >> 1;
                    if (s_roff[mid] <= o) lr = mid;
                    else hr = mid - 1;
                }
                tile_keys[o] = s_rtile[lr] + (o - s_roff[lr]);
                entries[o] = s_e[s_rlo[lr]];
            }
            base += tot;
        }
    }
}

// Tile ranges [start, end) from the sorted tile keys, empty tiles included
// (as an empty range at the position where they would start), so no clearing
// pass is needed: the thread at each boundary i (a change of key between i-1
// and i, or the two ends) closes the previous tile, writes the tiles strictly
// between the two keys and opens the next.  Keys >= T (never produced) count
// as T.
// Four boundaries per thread and pass, their key loads issued together (a
// pass over tens of millions of keys is otherwise bound by one load latency
// per boundary).
constexpr int RANGES_UNROLL = 4;

__global__ void ranges_kernel(const u32* keys, const u32* n_ptr, uint2* ranges, u32 T) {
    const u32 n = *n_ptr;
    const u64 stride = (u64)gridDim.x * blockDim.x;
    for (u64 base = (u64)blockIdx.x * blockDim.x + threadIdx.x; base <= n;
         base += RANGES_UNROLL * stride) {
        u32 kp[RANGES_UNROLL] = {}, kc[RANGES_UNROLL] = {};
        if (n > 0) {
#pragma unroll
            for (int j = 0; j < RANGES_UNROLL; ++j) {
                const u64 i = base + j * stride;
                const u32 ic = i < n ? (u32)i : n;   // position i, clamped to n
                kp[j] = load_or_zero(keys, ic - 1u + (ic == 0u ? 1u : 0u), n);
                kc[j] = load_or_zero(keys, ic, n);
            }
        }
#pragma unroll
        for (int j = 0; j < RANGES_UNROLL; ++j) {
            const u64 iw = base + j * stride;
            if (iw > n) break;
            const u32 i = (u32)iw;
            const int64_t prev = i == 0 ? -1 : (int64_t)(kp[j] < T ? kp[j] : T);
            const int64_t cur = i == n ? (int64_t)T : (int64_t)(kc[j] < T ? kc[j] : T);
            if (cur == prev) continue;
            if (prev >= 0 && prev < (int64_t)T) ranges[prev].y = i;
            for (int64_t t = prev + 1; t < cur && t < (int64_t)T; ++t) ranges[t] = make_uint2(i, i);
            if (cur < (int64_t)T) ranges[cur].x = i;
        }
    }
}

// ---- depth order inside each tile's list ------------------------------------
// Keys are (depth bits << 32 | entry): unique, so any correct sort gives the
// one order.  Lists are sorted by a bitonic network on keys held in registers
// (R per thread): by one wave up to 512 instances, by a 256-thread workgroup
// up to 2048; longer lists as workgroup-sorted runs of 2048 merged pairwise in
// global memory (each thread produces a contiguous piece of a merged run
// after locating its start on the merge path by binary search).
constexpr u32 SORT_WAVE_MAX = 512;
constexpr int SORT_LDS = 2048;
constexpr int SORT_THREADS = 256;

// value of lane ^ m (m a power of two below 64): quad permutations and a row
// rotation by 8 on the VALU, swizzles inside 32-lane halves, a lane
// permutation across the halves
__device__ __forceinline__ u32 xor_lanes(u32 v, int m) {
    switch (m) {
        case 1: return (u32)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
        case 2: return (u32)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
        case 4: return (u32)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
        case 8: return (u32)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);
        case 16: return (u32)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
        default: return (u32)__shfl_xor((int)v, m, 64);
    }
}

__device__ __forceinline__ u64 xor_lanes64(u64 x, int m) {
    return ((u64)xor_lanes((u32)(x >> 32), m) << 32) | xor_lanes((u32)x, m);
}

// One stage (merge size K, partner distance J) of the ascending bitonic
// network over the NT R keys of NT threads (one wave or a 256-thread
// workgroup), x[r] = element t R + r of thread t.  Partners at distance
// below R are registers of the thread; below 64 R, lanes of the same wave
// (DPP, swizzle or lane permutation); farther, other waves, through LDS
// (register-major, so the accesses are conflict-free).  The stages are
// template instances, so every register index is a constant.
template <int R, int NT, int K, int J>
__device__ __forceinline__ void bitonic_stage(u64 (&x)[R], u32 t, u64* lds) {
    if constexpr (J < R) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if ((r & J) == 0) {
                const int q = r | J;
                const bool up = ((t * R + r) & K) == 0;
                const u64 a = x[r], b = x[q];
                const bool sw = up ? (a > b) : (a < b);
                x[r] = sw ? b : a;
                x[q] = sw ? a : b;
            }
        }
    } else {
        constexpr int m = J / R;
        const bool lower = (t & m) == 0;
        u64 p[R];
        if constexpr (m < 64) {
            // all exchanges of the stage first, so their latencies overlap
#pragma unroll
            for (int r = 0; r < R; ++r) p[r] = xor_lanes64(x[r], m);
        } else {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) lds[r * NT + t] = x[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) p[r] = lds[r * NT + (t ^ m)];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool up = ((t * R + r) & K) == 0;
            // the lower element of an ascending pair keeps the minimum
            x[r] = ((x[r] < p[r]) == (lower == up)) ? x[r] : p[r];
        }
    }
    if constexpr (J > 1) bitonic_stage<R, NT, K, J / 2>(x, t, lds);
}

template <int R, int NT, int K>
__device__ __forceinline__ void bitonic_merges(u64 (&x)[R], u32 t, u64* lds) {
    bitonic_stage<R, NT, K, K / 2>(x, t, lds);
    if constexpr (K < NT * R) bitonic_merges<R, NT, 2 * K>(x, t, lds);
}

// keys of elements [0, L) of a list (1 <= L <= NT R), padded with the largest
// key.  The R entry loads are issued together (at clamped positions), then the
// R depth loads, so a thread waits twice instead of twice per key.
template <int R, int NT>
__device__ __forceinline__ void load_list_keys(u64 (&x)[R], const u32* ent, u32 L,
                                               const u32* depth_key, u32 E, u32 t) {
    u32 e[R], d[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const u32 i = t * R + r;
        e[r] = ent[i < L ? i : L - 1];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        e[r] = e[r] < E ? e[r] : E - 1;   // only for slots an overflowing frame left unwritten
        d[r] = depth_key[e[r]];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = t * R + r < L ? ((u64)d[r] << 32) | e[r] : ~0ull;
}

// sort one list of L <= NT R instances in place
template <int R, int NT>
__device__ __forceinline__ void group_sort_list(u32* ent, u32 L, const u32* depth_key, u32 E,
                                                u32 t, u64* lds) {
    u64 x[R];
    load_list_keys<R, NT>(x, ent, L, depth_key, E, t);
    bitonic_merges<R, NT, 2>(x, t, lds);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const u32 i = t * R + r;
        if (i < L) ent[i] = (u32)x[r];
    }
}

// sort one list of 2 .. 512 instances by one wave (lane = thread index in the wave)
__device__ __forceinline__ void wave_sort_short_list(u32* ent, u32 L, const u32* depth_key, u32 E,
                                                     u32 lane) {
    if (L <= 64) group_sort_list<1, 64>(ent, L, depth_key, E, lane, nullptr);
    else if (L <= 128) group_sort_list<2, 64>(ent, L, depth_key, E, lane, nullptr);
    else if (L <= 256) group_sort_list<4, 64>(ent, L, depth_key, E, lane, nullptr);
    else group_sort_list<8, 64>(ent, L, depth_key, E, lane, nullptr);
}

__device__ __forceinline__ u64 run_key(const u32* kh, const u32* kl, u32 i) {
    return ((u64)kh[i] << 32) | kl[i];
}

// One list longer than SORT_LDS, by the whole workgroup: runs of SORT_LDS
// sorted in registers into (sh0, sl0), then merged pairwise, ping-pong with
// (sh1, ent), where sh1 holds the list's tile ids, rewritten at the end.
__device__ void sort_long_list(u64* s, u32 tile, uint2 rg, const u32* depth_key, u32 E,
                               u32* inst_entry, u32* inst_tile, u32* sh0_all, u32* sl0_all) {
    const u32 L = rg.y - rg.x;
    const u32 t = threadIdx.x;
    u32* ent = inst_entry + rg.x;
    u32* ah = sh0_all + rg.x;
    u32* al = sl0_all + rg.x;
    u32* bh = inst_tile + rg.x;
    u32* bl = ent;
    constexpr int R = SORT_LDS / SORT_THREADS;
    for (u32 r0 = 0; r0 < L; r0 += SORT_LDS) {
        const u32 m = L - r0 < (u32)SORT_LDS ? L - r0 : (u32)SORT_LDS;
        u64 x[R];
        load_list_keys<R, SORT_THREADS>(x, ent + r0, m, depth_key, E, t);
        bitonic_merges<R, SORT_THREADS, 2>(x, t, s);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const u32 i = t * R + r;
            if (i < m) {
                ah[r0 + i] = (u32)(x[r] >> 32);
                al[r0 + i] = (u32)x[r];
            }
        }
    }
    __syncthreads();
    // merge passes, ping-pong between (ah, al) and (bh, bl)
    bool in_a = true;
    for (u32 w = SORT_LDS; w < L; w <<= 1) {
        const u32* srh = in_a ? ah : bh;
        const u32* srl = in_a ? al : bl;
        u32* dsh = in_a ? bh : ah;
        u32* dsl = in_a ? bl : al;
        for (u32 i0 = 0; i0 < L; i0 += 2 * w) {
            const u32 a0 = i0;
            const u32 a1 = i0 + w < L ? i0 + w : L;
            const u32 b1 = i0 + 2 * w < L ? i0 + 2 * w : L;
            const u32 na = a1 - a0, nb = b1 - a1, tot = na + nb;
            const u32 per = (tot + SORT_THREADS - 1) / SORT_THREADS;
            const u32 p0 = t * per;
            if (p0 >= tot) continue;
            const u32 p1 = p0 + per < tot ? p0 + per : tot;
            // merge path: how many of the first p0 outputs come from run A
            u32 lo = p0 > nb ? p0 - nb : 0, hi = p0 < na ? p0 : na;
            while (lo < hi) {
                const u32 mid = (lo + hi) >> 1;
                if (run_key(srh, srl, a0 + mid) < run_key(srh, srl, a1 + (p0 - mid - 1))) lo = mid + 1;
                else hi = mid;
            }
            // the two head keys stay in registers (an exhausted run reads as all
            // ones, above every key: depth bits are below the infinity pattern);
            // each step writes the smaller and loads the next of its run
            u32 ia = lo, ib = p0 - lo;
            u64 ka = ia < na ? run_key(srh, srl, a0 + ia) : ~0ull;
            u64 kb = ib < nb ? run_key(srh, srl, a1 + ib) : ~0ull;
            for (u32 p = p0; p < p1; ++p) {
                const bool take_a = ka < kb;
                const u64 k = take_a ? ka : kb;
                dsh[i0 + p] = (u32)(k >> 32);
                dsl[i0 + p] = (u32)k;
                if (take_a) {
                    ++ia;
                    ka = ia < na ? run_key(srh, srl, a0 + ia) : ~0ull;
                } else {
                    ++ib;
                    kb = ib < nb ? run_key(srh, srl, a1 + ib) : ~0ull;
                }
            }
        }
        __syncthreads();
        in_a = !in_a;
    }
    for (u32 j = t; j < L; j += SORT_THREADS) {
        if (in_a) ent[j] = al[j];
        bh[j] = tile;   // the tile ids the merge scratch overwrote
    }
}

// Every tile list in one launch: each 256-thread workgroup takes four tiles a
// grid apart (b, b + G, b + 2G, b + 3G), so the long lists of a dense image
// region, which sit on neighbouring tiles, land on different workgroups; wave
// w sorts tile b + w G if its list is short (up to 512 instances), then the
// workgroup sorts the longer lists among the four one after the other: in
// registers across its four waves up to SORT_LDS instances, beyond that as
// runs and merges.
constexpr u32 SORT_TILES = SORT_THREADS / 64;

__global__ void __launch_bounds__(SORT_THREADS) tile_sort_kernel(
    const uint2* ranges, u32 T, const u32* depth_key, u32 E, u32* inst_entry, u32* inst_tile,
    u32* sh0_all, u32* sl0_all) {
    __shared__ u64 s[SORT_LDS];
    {
        const u32 t = blockIdx.x + (threadIdx.x >> 6) * gridDim.x;
        const uint2 rg = t < T ? ranges[t] : make_uint2(0u, 0u);
        const u32 L = rg.y - rg.x;
        if (L > 1 && L <= SORT_WAVE_MAX)
            wave_sort_short_list(inst_entry + rg.x, L, depth_key, E, threadIdx.x & 63);
    }
    for (u32 k = 0; k < SORT_TILES; ++k) {
        const u32 tk = blockIdx.x + k * gridDim.x;
        const uint2 rg = tk < T ? ranges[tk] : make_uint2(0u, 0u);
        const u32 L = rg.y - rg.x;
        if (L <= SORT_WAVE_MAX) continue;
        if (L <= 1024)
            group_sort_list<4, SORT_THREADS>(inst_entry + rg.x, L, depth_key, E, threadIdx.x, s);
        else if (L <= (u32)SORT_LDS)
            group_sort_list<8, SORT_THREADS>(inst_entry + rg.x, L, depth_key, E, threadIdx.x, s);
        else
            sort_long_list(s, tk, rg, depth_key, E, inst_entry, inst_tile, sh0_all, sl0_all);
        __syncthreads();
    }
}

// Instance offsets and chunk starts of the visible entries in depth order
// (the epilogue of a scan of their tile counts, gathered through the sorted
// entry list); the totals were published by the entry-order scan.
struct PresortEpi {
    u32* inst_off;
    u32* chunk_start;
    u32 cap;
    __device__ void item(u32 slot, u32 tt, u32 off) const {
        inst_off[slot] = off;
        mark_chunks(chunk_start, cap, slot, off, tt);
    }
    __device__ void finish(u32) const {}
};

// First pass of the depth-order offsets scan: gathers the tile counts through
// the sorted entry list once (a random read per entry) into a contiguous array
// the second pass reads in order, and sums each partition.
__global__ void __launch_bounds__(GS_BLOCK) presort_gather_reduce_kernel(const u32* tt,
                                                                         const u32* sorted,
                                                                         const u32* n_dev,
                                                                         u32* tt_sorted, u32* part) {
    __shared__ u32 lds4[4];
    u32 beg, end;
    chunk_of(*n_dev, GS_SCAN_PARTS, blockIdx.x, beg, end);
    u32 s = 0;
    // four gathers per thread in flight per step
    for (u32 i = beg + threadIdx.x; i < end; i += 4 * GS_BLOCK) {
        u32 v[4];
        scan_in_n<4>(tt, sorted, i, GS_BLOCK, end, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i + j * GS_BLOCK < end) tt_sorted[i + j * GS_BLOCK] = v[j];
            s += v[j];
        }
    }
    u32 total;
    block_exclusive_scan(s, lds4, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// heavy-first order key: longer lists first (lists of 65535 instances or
// more tie), ties by tile id (stable sort); 16 bits, two radix passes
constexpr int TILE_WEIGHT_BITS = 16;
__global__ void tile_weight_kernel(const uint2* ranges, u32* keys, u32* vals, int T) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    constexpr u32 top = (1u << TILE_WEIGHT_BITS) - 1u;
    u32 len = ranges[t].y - ranges[t].x;
    if (len > top) len = top;
    keys[t] = top - len;
    vals[t] = (u32)t;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + GS_BLOCK - 1) / GS_BLOCK); }

}  // namespace

gs_status gs_launch_bin(gs_frame* f, hipStream_t s, bool heavy_first, bool presort,
                        bool balanced) {
    const int64_t E = f->E;
    u32* cnt = f->counters;
    if (E > 0) {
        // visible entries and instance offsets from the projection's tile
        // counts (read only, so rendering one projection twice repeats the work)
        u64* part = (u64*)f->scan_part;
        vis_reduce_kernel<<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(f->tiles_touched, (u32)E, part);
        GS_TRY(gs_check_launch("visible_reduce"));
        const VisEpi ve{f->visible, f->inst_off, f->chunk_start, cnt, (u32)f->cap, (u32)E,
                        f->depth_key, presort ? f->dkeys[0] : nullptr};
        vis_down_kernel<<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(f->tiles_touched, (u32)E, part, ve);
        GS_TRY(gs_check_launch("visible_scan"));
        if (presort) {
            // the visible entries in (depth bits, entry) order: a stable radix sort of
            // their depth keys over the entry-ordered list (four passes end in slot 0,
            // f->visible), then their instance offsets in that order
            u32* k[2] = {f->dkeys[0], f->dkeys[1]};
            u32* v[2] = {f->visible, f->dvals1};
            int slot = 0;
            GS_TRY(gs_radix_sort(k, v, cnt + 0, 0, E, 32, f->sort_scratch, &slot, s));
            if (slot != 0) return gs_fail(GS_ERR_HIP, "depth presort ended in the wrong buffer");
            // the depth keys are consumed: their first buffer holds the gathered counts
            u32* sp = f->scan_part;
            u32* tt_sorted = f->dkeys[0];
            presort_gather_reduce_kernel<<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(
                f->tiles_touched, f->visible, cnt + 0, tt_sorted, sp);
            GS_TRY(gs_check_launch("presort_gather"));
            const PresortEpi pe{f->inst_off, f->chunk_start, (u32)f->cap};
            scan_down_kernel<PresortEpi><<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(
                tt_sorted, nullptr, cnt + 0, 0, sp, pe);
            GS_TRY(gs_check_launch("presort_offsets"));
        }
        if (f->sigma3)
            emit_kernel<true><<<8192, GS_BLOCK, 0, s>>>(f->visible, f->inst_off, f->rect, f->splat,
                                                        f->d_views, f->n, cnt + 0, cnt + 5,
                                                        f->chunk_start, f->ikeys[0], f->ivals[0],
                                                        E, (u32)f->T);
        else
            emit_kernel<false><<<8192, GS_BLOCK, 0, s>>>(f->visible, f->inst_off, f->rect, f->splat,
                                                         f->d_views, f->n, cnt + 0, cnt + 5,
                                                         f->chunk_start, f->ikeys[0], f->ivals[0],
                                                         E, (u32)f->T);
        GS_TRY(gs_check_launch("emit"));
        // the per-tile sort orders each list by (depth bits, entry) afterwards, so
        // the first pass need not keep equal digits in order; after the depth
        // presort the tile sort must be stable throughout
        GS_TRY(gs_radix_sort(f->ikeys, f->ivals, cnt + 5, 0, f->cap, f->tile_bits, f->sort_scratch,
                             &f->isorted, s, balanced, !presort));
    } else {
        GS_TRY(gs_fill_u32(cnt, 0u, 6, s));
    }
    ranges_kernel<<<4096, GS_BLOCK, 0, s>>>(f->ikeys[f->isorted], cnt + 5, f->ranges, (u32)f->T);
    GS_TRY(gs_check_launch("ranges"));
    if (E > 0 && f->T > 0 && !presort) {
        const int o = f->isorted ^ 1;
        const unsigned sg = (unsigned)((f->T + SORT_TILES - 1) / SORT_TILES);
        tile_sort_kernel<<<sg, SORT_THREADS, 0, s>>>(f->ranges, (u32)f->T, f->depth_key, (u32)E,
                                                    f->ivals[f->isorted], f->ikeys[f->isorted],
                                                    f->ikeys[o], f->ivals[o]);
        GS_TRY(gs_check_launch("tile_sort"));
    }
    f->heavy_built = heavy_first;
    if (heavy_first) {
        tile_weight_kernel<<<blocks_for(f->T), GS_BLOCK, 0, s>>>(f->ranges, f->tkeys[0], f->tvals[0],
                                                                 f->T);
        GS_TRY(gs_check_launch("tile_weight"));
        GS_TRY(gs_radix_sort(f->tkeys, f->tvals, nullptr, (u32)f->T, f->T, TILE_WEIGHT_BITS,
                             f->sort_scratch, &f->tsorted, s));
    }
    return GS_OK;
}
