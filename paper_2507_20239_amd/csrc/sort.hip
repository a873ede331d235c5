// Prefix sums and stable LSD radix sort for wave64 (gfx950).
//
// Both work on a length that may live in device memory, so a step can be
// enqueued (or captured into a graph) without reading counts on the host:
// the grid is a fixed number of partitions and every workgroup derives its
// chunk from the device length.
//
// Radix sort: 8-bit digits; per pass, per-workgroup digit counts, an
// exclusive scan of the count matrix and a stable scatter.  Keys are ranked
// inside a workgroup with a wave-level multi-split: one ballot per digit bit
// gives each lane the mask of lanes holding the same digit, the popcount below
// the lane is its rank within the item, per-wave running counters in LDS
// order successive items, and a 4-wave exclusive scan orders the waves.  A
// pass that may reorder equal digits ranks each key with one LDS add instead.
#include "gs_internal.h"

namespace {

constexpr int RADIX_ITEMS = 8;                       // keys per lane per sub-batch
constexpr int RADIX_SUB = GS_BLOCK * RADIX_ITEMS;    // 2048 keys per sub-batch

__global__ void fill_u32_kernel(u32* p, u32 value, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

__global__ void __launch_bounds__(GS_BLOCK) scan_reduce_kernel(const u32* in, const u32* gather,
                                                               const u32* n_dev, u32 n_host,
                                                               u32* part) {
    __shared__ u32 lds4[4];
    u32 beg, end;
    chunk_of(dev_len(n_dev, n_host), GS_SCAN_PARTS, blockIdx.x, beg, end);
    u32 s = 0;
    // four values per thread in flight per step
    for (u32 i = beg + threadIdx.x; i < end; i += 4 * GS_BLOCK) {
        u32 v[4];
        scan_in_n<4>(in, gather, i, GS_BLOCK, end, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) s += v[j];
    }
    u32 total;
    block_exclusive_scan(s, lds4, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// ---- Radix pass: per-workgroup digit counts (digit-major matrix [256][G]),
// a scan of each digit's row over the workgroups plus the digit totals, and a
// stable scatter that adds the digit bases (which gives every workgroup the
// start of each of its digit runs).  Workgroup counts could also be combined
// by a chained (decoupled look-back) scan or by each workgroup summing the
// rows before it; both were measured to be latency-bound on this part
// (device-scope loads cross the XCDs).  The scatter reorders each 2048-key
// sub-batch by digit in LDS first, so consecutive lanes write consecutive
// addresses of a digit run (coalesced) instead of scattering 4-byte stores.

__global__ void __launch_bounds__(GS_BLOCK) sort_count_kernel(const u32* __restrict__ keys,
                                                              const u32* n_dev, u32 n_host,
                                                              int shift, int bits, u32* counts) {
    __shared__ u32 h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    u32 beg, end;
    chunk_of(dev_len(n_dev, n_host), gridDim.x, blockIdx.x, beg, end);
    const u32 mask = (1u << bits) - 1u;
    const u32 lane = threadIdx.x & 63u;
    const u64 above = lane < 63 ? ~0ull << (lane + 1) : 0ull;   // lanes above this one
    // Counting needs no order among equal digits: one LDS add per run of equal
    // digits in consecutive lanes, by the run's first lane (key streams here
    // are locally coherent: a footprint's tiles, a tile group's high digit),
    // and the LDS serialises only the equal digits that remain in a wave.
    for (u32 base = beg; base < end; base += 8 * GS_BLOCK) {
        u32 k[8];
        // eight keys per thread loaded together (the loop is bound by load latency)
#pragma unroll
        for (int j = 0; j < 8; ++j) k[j] = load_or_zero(keys, base + j * GS_BLOCK + threadIdx.x, end);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool valid = base + j * GS_BLOCK + threadIdx.x < end;   // a prefix of the wave
            const u32 d = valid ? (k[j] >> shift) & mask : 0xffffffffu;
            const u32 prev = (u32)__shfl_up((int)d, 1, 64);
            const bool head = valid && (lane == 0 || d != prev);
            // a run ends where the next one starts or the valid lanes end
            const u64 stops = __ballot(head) | ~__ballot(valid);
            if (head) {
                const u64 nxt = stops & above;
                const u32 len = (nxt ? (u32)__builtin_ctzll(nxt) : 64u) - lane;
                atomicAdd(&h[d], len);
            }
        }
    }
    __syncthreads();
    counts[(u64)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of the digit's row of workgroup
// counts (counts[d][0..G), G <= 2048, in place) and the digit's total.  The
// scatter adds the digit bases (an exclusive scan of the 256 totals, which
// every scatter workgroup computes for itself), so a pass is three launches.
__global__ void __launch_bounds__(GS_BLOCK) sort_rowscan_kernel(u32* counts, u32 G, u32* dtot) {
    __shared__ u32 lds4[4];
    u32* row = counts + (u64)blockIdx.x * G;
    const u32 i0 = threadIdx.x * 8;
    u32 v[8];
    u32 sum = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = i0 + j < G ? row[i0 + j] : 0u;
        sum += v[j];
    }
    u32 total;
    u32 ex = block_exclusive_scan(sum, lds4, total);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (i0 + j < G) row[i0 + j] = ex;
        ex += v[j];
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = total;
}

__global__ void __launch_bounds__(GS_BLOCK) sort_scatter_kernel(
    const u32* __restrict__ kin, const u32* __restrict__ vin, u32* __restrict__ kout,
    u32* __restrict__ vout, const u32* n_dev, u32 n_host, int shift, int bits,
    const u32* __restrict__ offs, const u32* __restrict__ dtot, int unstable) {
    __shared__ u32 whist[4][256];
    __shared__ u32 s_base[256];    // global start of each digit's run for the next sub-batch
    __shared__ u32 s_local[256];   // start of each digit inside the sub-batch
    __shared__ u32 s_key[RADIX_SUB], s_val[RADIX_SUB];
    __shared__ u32 lds4[4];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const u32 n = dev_len(n_dev, n_host);
    {
        u32 all;
        const u32 dbase = block_exclusive_scan(dtot[tid], lds4, all);
        s_base[tid] = dbase + offs[(u64)tid * gridDim.x + blockIdx.x];
    }
    u32 beg, end;
    chunk_of(n, gridDim.x, blockIdx.x, beg, end);
    const u32 mask = (1u << bits) - 1u;
    for (u32 sub = beg; sub < end; sub += RADIX_SUB) {
        for (int j = lane; j < 256; j += 64) whist[w][j] = 0;
        __syncthreads();
        u32 k[RADIX_ITEMS], v[RADIX_ITEMS], r[RADIX_ITEMS];
        // every item's key and value loaded before any is ranked: sixteen loads in
        // flight per thread instead of one round trip per item
#pragma unroll
        for (int i = 0; i < RADIX_ITEMS; ++i) {
            const u32 idx = sub + (u32)(w * 64 * RADIX_ITEMS + i * 64 + lane);
            k[i] = load_or_zero(kin, idx, end);
            v[i] = load_or_zero(vin, idx, end);
        }
#pragma unroll
        for (int i = 0; i < RADIX_ITEMS; ++i) {
            const u32 idx = sub + (u32)(w * 64 * RADIX_ITEMS + i * 64 + lane);
            const bool valid = idx < end;   // a prefix of the wave
            const u32 d = (k[i] >> shift) & mask;
            if (unstable) {
                // any order among equal digits: one LDS add per key takes its place
                r[i] = valid ? atomicAdd(&whist[w][d], 1u) : 0u;
                continue;
            }
            // lanes whose digit differs in some bit: a lane with bit b set
            // differs from the lanes without it (~ballot), else from those with it
            u64 differ = ~__ballot(valid);
            for (int b = 0; b < bits; ++b) {
                const u32 sb = (u32)((int)(d << (31 - b)) >> 31);   // bit b as 0 or all ones
                differ |= __ballot(sb != 0u) ^ (((u64)sb << 32) | sb);
            }
            const u64 peers = ~differ;
            const u32 lo = popc_below(peers);
            const u32 cnt = (u32)__popcll(peers);
            u32 prior = 0;
            if (valid) prior = whist[w][d];
            r[i] = prior + lo;
            // the highest lane of each digit group advances the wave counter
            if (valid && lo == cnt - 1u) whist[w][d] = prior + cnt;
        }
        __syncthreads();
        const u32 c0 = whist[0][tid], c1 = whist[1][tid], c2 = whist[2][tid], c3 = whist[3][tid];
        const u32 tot = c0 + c1 + c2 + c3;
        u32 subtotal;
        const u32 loc = block_exclusive_scan(tot, lds4, subtotal);
        s_local[tid] = loc;
        whist[0][tid] = loc;
        whist[1][tid] = loc + c0;
        whist[2][tid] = loc + c0 + c1;
        whist[3][tid] = loc + c0 + c1 + c2;
        __syncthreads();
        // place the sub-batch in LDS in (digit, rank) order
#pragma unroll
        for (int i = 0; i < RADIX_ITEMS; ++i) {
            const u32 idx = sub + (u32)(w * 64 * RADIX_ITEMS + i * 64 + lane);
            if (idx < end) {
                const u32 pos = whist[w][(k[i] >> shift) & mask] + r[i];
                s_key[pos] = k[i];
                s_val[pos] = v[i];
            }
        }
        __syncthreads();
        // write out: position i of the reordered sub-batch goes to its digit run
        for (u32 i = (u32)tid; i < subtotal; i += GS_BLOCK) {
            const u32 key = s_key[i];
            const u32 dd = (key >> shift) & mask;
            const u32 pos = s_base[dd] + (i - s_local[dd]);
            if (pos < n) {
                kout[pos] = key;
                vout[pos] = s_val[i];
            }
        }
        __syncthreads();
        s_base[tid] += tot;
    }
}

// One workgroup per 4096 slots of capacity, at most 7 per CU (the scatter's
// LDS allows seven per CU; its loop is bound by load latency, so a full CU
// hides more of it): 1792 on 256 CUs.
constexpr int64_t SORT_MAX_BLOCKS = 1792;

unsigned sort_blocks(int64_t capacity) {
    int64_t g = (capacity + 4095) / 4096;
    if (g < 1) g = 1;
    if (g > SORT_MAX_BLOCKS) g = SORT_MAX_BLOCKS;
    return (unsigned)g;
}

}  // namespace

uint64_t gs_radix_scratch_bytes(int64_t capacity, int bits) {
    (void)bits;
    return 4 * 256 * (uint64_t)sort_blocks(capacity) + 4 * (GS_SCAN_PARTS + 8);
}

gs_status gs_fill_u32(u32* p, u32 value, int64_t count, hipStream_t s) {
    if (count <= 0) return GS_OK;
    int64_t blocks = (count + GS_BLOCK - 1) / GS_BLOCK;
    if (blocks > 4096) blocks = 4096;
    fill_u32_kernel<<<(unsigned)blocks, GS_BLOCK, 0, s>>>(p, value, count);
    return gs_check_launch("fill_u32");
}

gs_status gs_scan_reduce(const u32* in, const u32* gather, const u32* n_dev, u32 n_host, u32* part,
                         hipStream_t s) {
    scan_reduce_kernel<<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(in, gather, n_dev, n_host, part);
    return gs_check_launch("scan_reduce");
}

gs_status gs_scan_exclusive(const u32* in, u32* out, const u32* n_dev, u32 n_host, u32* total,
                            u32* part, hipStream_t s, const u32* gather) {
    GS_TRY(gs_scan_reduce(in, gather, n_dev, n_host, part, s));
    ScanStore epi{out, total};
    scan_down_kernel<ScanStore><<<GS_SCAN_PARTS, GS_BLOCK, 0, s>>>(in, gather, n_dev, n_host, part,
                                                                   epi);
    return gs_check_launch("scan_exclusive");
}

gs_status gs_radix_sort(u32* k[2], u32* v[2], const u32* n_dev, u32 n_host, int64_t capacity,
                        int bits, void* scratch, int* slot, hipStream_t s, bool balanced,
                        bool unstable_first) {
    const unsigned G = sort_blocks(capacity);
    u32* counts = (u32*)scratch;
    u32* part = counts + 256 * (uint64_t)G;
    int cur = 0;
    // the same number of passes either way; balanced digits split the bits evenly
    const int passes = (bits + 7) / 8;
    const int width = balanced ? (bits + passes - 1) / passes : 8;
    for (int shift = 0; shift < bits; shift += width) {
        const int b = (bits - shift) < width ? (bits - shift) : width;
        sort_count_kernel<<<G, GS_BLOCK, 0, s>>>(k[cur], n_dev, n_host, shift, b, counts);
        GS_TRY(gs_check_launch("sort_count"));
        sort_rowscan_kernel<<<256, GS_BLOCK, 0, s>>>(counts, G, part);
        GS_TRY(gs_check_launch("sort_rowscan"));
        sort_scatter_kernel<<<G, GS_BLOCK, 0, s>>>(k[cur], v[cur], k[cur ^ 1], v[cur ^ 1], n_dev,
                                                   n_host, shift, b, counts, part,
                                                   unstable_first && shift == 0 ? 1 : 0);
        GS_TRY(gs_check_launch("sort_scatter"));
        cur ^= 1;
    }
    *slot = cur;
    return GS_OK;
}
