// gs_bin_sort kernels: scan of tiles_touched, (tile, depth) key emission,
// onesweep LSD radix sort (8-bit digits, decoupled look-back across
// partitions) and per-tile ranges.
//
// Onesweep on CDNA4: a partition of 4096 keys per 512-thread workgroup (eight
// wave64, 8 keys per lane), so that a frame's ~1M keys occupy every CU.  The
// digit counts of every pass come from the emission kernel.  Ranks inside a wave come from eight ballots per
// key (the lanes holding the same digit), so ranking is stable: stripes are
// processed in index order and lanes inside a stripe are in index order.
// A persistent grid takes partitions by an atomic ticket, so a workgroup
// only ever waits for partitions that a running workgroup already holds
// (forward progress); the grid is sized to the machine, not the capacity.  Each partition publishes per-digit counts in one 32-bit word
// (2 flag bits + 30 count bits) with agent-scope atomics, because the eight
// XCDs have private L2s.  The look-back reads 64 predecessor statuses per
// round trip (all partitions of a pass run at once on this size of problem,
// so a one-at-a-time walk would serialise); a lane that meets an unpublished
// predecessor sleeps briefly and polls again.  The scatter is staged through
// LDS so that each digit's run is written contiguously.
#include "gs_internal.hpp"

namespace gs {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;  // 4096 instances per block

constexpr int kSortBlock = 512;
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kMinSortItems = 8;                    // partitions of 4096 or 8192 keys (tunable)
constexpr int kMinSortPart = kSortBlock * kMinSortItems;
constexpr int kEmitGrid = 1024;  // emission workgroups at most (grid-stride over scan tiles beyond)
constexpr int kBucketGrid = 256;  // emission workgroups of the bucket path (rows of the tile counters)
constexpr int64_t kBucketMaxTiles = 4096;  // the bucket path serves up to this many tiles (all views)
constexpr int kRadixBits = 8;
constexpr int kBins = 1 << kRadixBits;
constexpr int kMaxPasses = 8;
constexpr int kHistStride = kBins + 1;  // per-pass difference array of the digit counts
constexpr int kHistRows = 16;           // partial histogram rows left by hist_reduce_kernel
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagIncl = 2u << 30;
constexpr uint32_t kCountMask = (1u << 30) - 1u;

// ---------------------------------------------------------------------------
// fill (used instead of memset nodes so a captured graph replays correctly)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n, int64_t stride) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

// zeroes two buffers in one launch
__global__ void __launch_bounds__(256) clear2_kernel(uint32_t *a, int64_t na, uint32_t *b, int64_t nb, int64_t stride) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < na; i += stride) a[i] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nb; i += stride) b[i] = 0u;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    return launch_kernel(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), s, p, v, n, blocks * 256);
}

// ---------------------------------------------------------------------------
// scan of tiles_touched (reduce, scan of block sums, downsweep)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t block_reduce_u64(uint64_t v, uint64_t *s_tmp) {
    // wave reduction then across the four waves
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) s_tmp[w] = v;
    __syncthreads();
    uint64_t t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kScanBlock / 64; ++k) t += s_tmp[k];
    return t;  // valid in thread 0
}

__global__ void __launch_bounds__(kScanBlock) scan_reduce_kernel(const uint32_t *tt, int64_t n, uint64_t *part) {
    __shared__ uint64_t s_tmp[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k * kScanBlock + threadIdx.x;
        if (i < n) acc += tt[i];
    }
    const uint64_t t = block_reduce_u64(acc, s_tmp);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// one workgroup of 1024 threads: exclusive scan of the block sums in place;
// writes K and the overflow flag
__global__ void __launch_bounds__(1024) scan_partials_kernel(uint64_t *part, int64_t nparts, int64_t capacity,
                                                             int64_t *d_num, int32_t *d_overflow) {
    __shared__ uint64_t s[1024];
    uint64_t carry = 0;
    for (int64_t base = 0; base < nparts; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const uint64_t v = (i < nparts) ? part[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint64_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nparts) part[i] = carry + s[threadIdx.x] - v;
        carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *d_num = (int64_t)carry;
        *d_overflow = ((int64_t)carry > capacity) ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// key emission
// ---------------------------------------------------------------------------
// Digit counts are kept as difference arrays (count of digit d = sum of
// diff[0..d]) so that a run of consecutive digits costs two updates.
__device__ __forceinline__ void hist_add(uint32_t *h, uint32_t d, uint32_t c) {
    atomicAdd(&h[d], c);
    atomicSub(&h[d + 1], c);
}

// adds the tile digits of one rect row (tiles [t0, t0 + w)) to the per-pass
// difference arrays of the tile bytes (passes 4 .. passes-1)
__device__ __forceinline__ void hist_add_row(uint32_t (*h)[kHistStride], int passes, uint64_t t0, uint32_t w) {
    // lowest tile byte: w consecutive digits, wrapping mod 256
    {
        uint32_t *hp = h[4];
        const uint32_t full = w >> 8, rem = w & 255u, lo = (uint32_t)(t0 & 255u);
        if (full) {  // every digit, `full` times
            atomicAdd(&hp[0], full);
            atomicSub(&hp[256], full);
        }
        if (rem) {
            if (lo + rem <= 256u) {
                atomicAdd(&hp[lo], 1u);
                atomicSub(&hp[lo + rem], 1u);
            } else {
                atomicAdd(&hp[lo], 1u);
                atomicSub(&hp[256], 1u);
                atomicAdd(&hp[0], 1u);
                atomicSub(&hp[lo + rem - 256u], 1u);
            }
        }
    }
    // higher tile bytes: constant over runs of 256^b tiles
    for (int p = 5; p < passes; ++p) {
        const int sh = 8 * (p - 4);
        uint64_t t = t0;
        const uint64_t end = t0 + w;
        while (t < end) {
            uint64_t seg = ((t >> sh) + 1) << sh;
            if (seg > end) seg = end;
            hist_add(h[p], (uint32_t)(t >> sh) & 255u, (uint32_t)(seg - t));
            t = seg;
        }
    }
}

// Key emission, fused with the downsweep of the scan of tiles_touched and
// with the digit histograms of every sort pass.  A workgroup of 1024 threads
// takes a scan tile of 4096 instances (thread t owns 4 consecutive ones) and
// turns the block-local scan plus the tile's global prefix into each
// instance's first key.  Each wave (256 instances) compacts its live
// instances -- visible, with keys below the capacity -- into LDS, in index
// order, and its lanes then work through that list together: tile rect,
// histogram updates (the four depth bytes once per instance with weight
// tiles_touched, the tile bytes per rect row), key layout.  The keys of a
// wave fill one contiguous stretch of the output, written with coalesced
// stores: lane j takes keys j, j + 64, ... and finds the owning instance by
// a binary search over the list's key starts.  Each workgroup leaves its
// histograms as one row of `rows` (plain stores) for hist_reduce_kernel.
constexpr int kEmitBlock = 1024;
constexpr int kEmitItems = kScanTile / kEmitBlock;  // 4 instances per thread
constexpr int kEmitWaves = kEmitBlock / 64;
constexpr int kWaveInst = 64 * kEmitItems;          // 256 instances per wave
constexpr int kLdsTiles = 4096;                     // LDS words for tile counters / digit histograms
static_assert(kLdsTiles >= kMaxPasses * kHistStride, "the LDS buffer also holds the digit histograms");
static_assert(kBucketMaxTiles <= kLdsTiles, "bucket tile counters live in LDS");

enum EmitMode { kEmitSortKeys = 0, kEmitCountTiles = 1, kEmitScatterTiles = 2 };

struct EmitArgs {
    const uint32_t *tt;
    const uint64_t *part;
    const float4 *rec;
    int64_t n, n_tiles_scan, capacity, n_blocks;
    int TX, TY;
    // kEmitSortKeys: keys, values and the digit histograms of every pass
    uint64_t *keys;
    uint32_t *vals;
    int passes;
    uint32_t *rows;  // [grid][passes * 257]
    // kEmitCountTiles / kEmitScatterTiles: per-workgroup tile counters
    uint32_t *tile_cnt;          // [n_tiles][grid]: counts, then running offsets within the tile
    const uint32_t *tile_start;  // [n_tiles]: first key of each tile
    uint64_t *bucket;            // [capacity]: (depth bits << 32) | instance, grouped by tile
    int64_t n_tiles;
    const int32_t *d_overflow;
};

template <int MODE>
__global__ void __launch_bounds__(kEmitBlock) emit_kernel(const EmitArgs A) {
    // digit histograms (sort keys) or, for up to kLdsTiles tiles, the
    // workgroup's tile counters (count / scatter)
    __shared__ uint32_t s_aux[kLdsTiles];
    uint32_t(*s_h)[kHistStride] = reinterpret_cast<uint32_t(*)[kHistStride]>(s_aux);
    __shared__ uint64_t s_wsum[kEmitWaves];
    // per wave, per list entry: staged record, then the emission layout
    __shared__ uint32_t s_a0[kEmitWaves][kWaveInst];  // u bits          -> rect origin x0 | y0 << 16
    __shared__ uint32_t s_a1[kEmitWaves][kWaveInst];  // v bits          -> rect width
    __shared__ uint32_t s_a2[kEmitWaves][kWaveInst];  // depth bits
    __shared__ uint32_t s_a3[kEmitWaves][kWaveInst];  // radius          -> first tile of the view
    __shared__ uint32_t s_a4[kEmitWaves][kWaveInst];  // view
    __shared__ uint32_t s_a5[kEmitWaves][kWaveInst];  // instance index
    __shared__ uint32_t s_a6[kEmitWaves][kWaveInst];  // first key, relative to the wave's first
    __shared__ uint32_t s_a7[kEmitWaves][kWaveInst];  // tiles_touched
    if (MODE == kEmitScatterTiles && *A.d_overflow) return;  // nothing consistent to scatter
    const uint32_t *tt = A.tt;
    const float4 *rec = A.rec;
    const int64_t n = A.n, capacity = A.capacity;
    const int TX = A.TX, TY = A.TY, passes = A.passes;
    if (MODE == kEmitSortKeys)
        for (int k = threadIdx.x; k < kMaxPasses * kHistStride; k += kEmitBlock) s_aux[k] = 0u;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // tile counters in HBM are tile-major: tile t's counts of all workgroups are one row
    uint32_t *my_cnt = A.tile_cnt + blockIdx.x;
    const int64_t cs = A.n_blocks;  // row stride
    // count / scatter: the tile counters live in LDS (at most kLdsTiles tiles)
    if (MODE == kEmitCountTiles)
        for (int k = threadIdx.x; k < A.n_tiles; k += kEmitBlock) s_aux[k] = 0u;
    if (MODE == kEmitScatterTiles)  // this workgroup's first slot in every bucket
        for (int k = threadIdx.x; k < A.n_tiles; k += kEmitBlock) s_aux[k] = A.tile_start[k] + my_cnt[k * cs];
    for (int64_t tile = blockIdx.x; tile < A.n_tiles_scan; tile += A.n_blocks) {  // uniform per workgroup
        const int64_t base = tile * kScanTile + (int64_t)threadIdx.x * kEmitItems;
        uint32_t v[kEmitItems];
        if (base + kEmitItems <= n) {  // one 16-B load (tt is 16-B aligned: caller-owned allocation)
            const uint4 q = *reinterpret_cast<const uint4 *>(tt + base);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
#pragma unroll
            for (int k = 0; k < kEmitItems; ++k) v[k] = (base + k < n) ? tt[base + k] : 0u;
        }
        // wave-level inclusive scan of the per-thread sums (fits 32 bits:
        // 256 instances of at most 2^22 tiles), then across the waves in 64 bits
        uint32_t incl = v[0] + v[1] + v[2] + v[3];
        const uint32_t own = incl;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        const uint32_t wave_total = __shfl(incl, 63, 64);
        // sort keys go to the wave's stretch of the key array (first key kw,
        // nothing past the capacity); the bucket modes place keys by tile
        // counters instead and scatter only when the total fits
        int64_t kw = 0, room = INT64_MAX;
        if (MODE == kEmitSortKeys) {
            if (lane == 0) s_wsum[wave] = wave_total;
            __syncthreads();
            uint64_t wave_excl = 0;
            for (int k = 0; k < wave; ++k) wave_excl += s_wsum[k];
            kw = (int64_t)(A.part[tile] + wave_excl);
            room = capacity - kw;
        }
        // live instances of the lane and their place in the wave's list
        uint32_t start[kEmitItems];
        uint32_t live_mask = 0u;
        {
            uint32_t run = incl - own;
#pragma unroll
            for (int k = 0; k < kEmitItems; ++k) {
                start[k] = run;
                if (v[k] && (int64_t)run < room) live_mask |= 1u << k;
                run += v[k];
            }
        }
        const uint32_t cnt = __popc(live_mask);
        uint32_t pos = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(pos, off, 64);
            if (lane >= off) pos += y;
        }
        const uint32_t n_live = __shfl(pos, 63, 64);
        pos -= cnt;
        // stage the live instances' records (all loads in flight together)
        float4 q0[kEmitItems];
        uint32_t view[kEmitItems];
#pragma unroll
        for (int k = 0; k < kEmitItems; ++k)
            if (live_mask & (1u << k)) {
                q0[k] = rec[3 * (base + k)];
                view[k] = (uint32_t)__float_as_int(rec[3 * (base + k) + 2].w);
            }
#pragma unroll
        for (int k = 0; k < kEmitItems; ++k)
            if (live_mask & (1u << k)) {
                s_a0[wave][pos] = __float_as_uint(q0[k].x);
                s_a1[wave][pos] = __float_as_uint(q0[k].y);
                s_a2[wave][pos] = __float_as_uint(q0[k].z);
                s_a3[wave][pos] = __float_as_uint(q0[k].w);
                s_a4[wave][pos] = view[k];
                s_a5[wave][pos] = (uint32_t)(base + k);
                s_a6[wave][pos] = start[k];
                s_a7[wave][pos] = v[k];
                ++pos;
            }
        __builtin_amdgcn_wave_barrier();
        // the list, lanes together: rect, histograms, emission layout
        for (uint32_t e = lane; e < n_live; e += 64) {
            const float u = __uint_as_float(s_a0[wave][e]), vv = __uint_as_float(s_a1[wave][e]);
            const uint32_t depth_bits = s_a2[wave][e];
            const Rect R = tile_rect(u, vv, (int)s_a3[wave][e], TX, TY);
            const uint64_t tbase = (uint64_t)s_a4[wave][e] * (uint64_t)(TX * TY);
            const uint32_t t = s_a7[wave][e];
            if (MODE == kEmitSortKeys) {
#pragma unroll
                for (int p = 0; p < 4; ++p) hist_add(s_h[p], (depth_bits >> (8 * p)) & 255u, t);
                for (int ty = R.y0; ty < R.y1; ++ty)
                    hist_add_row(s_h, passes, tbase + (uint64_t)(ty * TX + R.x0), (uint32_t)(R.x1 - R.x0));
            }
            s_a0[wave][e] = (uint32_t)R.x0 | ((uint32_t)R.y0 << 16);
            s_a1[wave][e] = (uint32_t)(R.x1 - R.x0);
            s_a3[wave][e] = (uint32_t)tbase;
        }
        __builtin_amdgcn_wave_barrier();
        // the wave's keys: list starts increase strictly, so the owner of key
        // j is the last entry whose start is <= j
        if (n_live) {
            const uint32_t lim = (int64_t)wave_total < room ? wave_total : (uint32_t)room;
            for (uint32_t j = lane; j < lim; j += 64) {
                int lo = 0, hi = (int)n_live - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_a6[wave][mid] <= j) lo = mid;
                    else hi = mid - 1;
                }
                const uint32_t rel = j - s_a6[wave][lo];
                const uint32_t w = s_a1[wave][lo], xy = s_a0[wave][lo];
                const uint32_t ty = (xy >> 16) + rel / w, tx = (xy & 0xFFFFu) + rel % w;
                const uint32_t tg = s_a3[wave][lo] + ty * (uint32_t)TX + tx;  // tile across all views
                if (MODE == kEmitSortKeys) {
                    const int64_t k = kw + (int64_t)j;
                    A.keys[k] = ((uint64_t)tg << 32) | (uint64_t)s_a2[wave][lo];
                    A.vals[k] = s_a5[wave][lo];
                } else if (MODE == kEmitCountTiles) {
                    atomicAdd(s_aux + tg, 1u);
                } else {
                    const uint32_t slot = atomicAdd(s_aux + tg, 1u);
                    A.bucket[slot] = ((uint64_t)s_a2[wave][lo] << 32) | (uint64_t)s_a5[wave][lo];
                }
            }
        }
        __syncthreads();  // s_wsum and the lists are reused by the next tile
    }
    if (MODE == kEmitSortKeys) {
        __syncthreads();
        uint32_t *row = A.rows + (size_t)blockIdx.x * passes * kHistStride;
        for (int k = threadIdx.x; k < passes * kHistStride; k += kEmitBlock) row[k] = s_aux[k];
    }
    if (MODE == kEmitCountTiles) {
        __syncthreads();
        for (int k = threadIdx.x; k < A.n_tiles; k += kEmitBlock) my_cnt[k * cs] = s_aux[k];
    }
}

// Partial sums of the emission rows: part[ry][c] = sum of rows[r][c] over the
// ry-th sixteenth of the rows (64 columns x 4 row lanes per workgroup).  The
// sort passes add up the kHistRows partials of their own digit column.
__global__ void __launch_bounds__(256) hist_reduce_kernel(const uint32_t *rows, int n_rows, int n_cols,
                                                          uint32_t *part /*[kHistRows][n_cols]*/) {
    __shared__ uint32_t s_part[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int rl = threadIdx.x >> 6;
    const int per = (n_rows + kHistRows - 1) / kHistRows;
    const int r0 = blockIdx.y * per, r1 = min(n_rows, r0 + per);
    uint32_t acc = 0u;
    if (c < n_cols)
        for (int r = r0 + rl; r < r1; r += 4) acc += rows[(size_t)r * n_cols + c];
    s_part[rl][threadIdx.x & 63] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && c < n_cols)
        part[(size_t)blockIdx.y * n_cols + c] =
            s_part[0][threadIdx.x] + s_part[1][threadIdx.x] + s_part[2][threadIdx.x] + s_part[3][threadIdx.x];
}

// ---------------------------------------------------------------------------
// onesweep radix sort
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t sort_count(const int64_t *d_num, int64_t capacity) {
    const int64_t k = *d_num;
    return k < capacity ? k : capacity;
}

template <int ITEMS, int LOOKBACK>
__global__ void __launch_bounds__(kSortBlock) onesweep_kernel(const uint64_t *__restrict__ keys_in,
                                                              const uint32_t *__restrict__ vals_in,
                                                              uint64_t *__restrict__ keys_out,
                                                              uint32_t *__restrict__ vals_out, const int64_t *d_num,
                                                              int64_t capacity, int shift,
                                                              const uint32_t *digit_base /*[256]*/,
                                                              uint32_t *status /*[parts][256]*/, uint32_t *ticket,
                                                              const int32_t *d_overflow) {
    __shared__ uint32_t s_part, s_next;
    __shared__ uint32_t s_wh[kSortWaves][kBins];  // per-wave digit counts -> prefix across waves
    __shared__ uint32_t s_local[kBins];           // block-local exclusive digit start
    __shared__ uint32_t s_glob[kBins];            // global start of the digit for this partition
    __shared__ uint32_t s_scan[kBins];
    __shared__ uint32_t s_base[kBins];            // global start of each digit in this pass
    __shared__ uint64_t s_keys[kSortBlock * ITEMS];
    __shared__ uint32_t s_vals[kSortBlock * ITEMS];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (*d_overflow) return;  // keys beyond the capacity were dropped: nothing consistent to sort
    const int64_t K = sort_count(d_num, capacity);
    // the first ticket and the digit bases, in flight together
    if (tid == 0) s_part = atomicAdd(ticket, 1u);
    if (tid < kBins) s_base[tid] = digit_base[tid];
    for (int k = tid; k < kSortWaves * kBins; k += kSortBlock) (&s_wh[0][0])[k] = 0u;
    __syncthreads();
    uint32_t part = s_part;
    // persistent: take partitions in ticket order until none is left
    while (true) {
        const int64_t start = (int64_t)part * (kSortBlock * ITEMS);
        if (start >= K) return;  // uniform across the workgroup

        uint64_t key[ITEMS];
        uint32_t val[ITEMS];
        uint32_t rank[ITEMS];
        uint32_t dig[ITEMS];
        // all loads first (independent, in flight together), then the ranking
        // (whose LDS fences would otherwise serialise one load per stripe)
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t idx = start + (int64_t)wave * (ITEMS * 64) + j * 64 + lane;
            const bool valid = idx < K;
            key[j] = valid ? keys_in[idx] : ~0ull;
            val[j] = valid ? vals_in[idx] : 0u;
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t idx = start + (int64_t)wave * (ITEMS * 64) + j * 64 + lane;
            const bool valid = idx < K;
            const uint32_t d = (uint32_t)(key[j] >> shift) & (kBins - 1);
            dig[j] = valid ? d : 0xFFFFFFFFu;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            uint32_t r = 0;
            if (valid) {
                const uint32_t below = __popcll(peers & lt_mask);
                const uint32_t prev = s_wh[wave][d];
                r = prev + below;
                __builtin_amdgcn_wave_barrier();
                if (below == 0) s_wh[wave][d] = prev + (uint32_t)__popcll(peers);
            } else {
                __builtin_amdgcn_wave_barrier();
            }
            __builtin_amdgcn_wave_barrier();
            rank[j] = r;
        }
        __syncthreads();
        uint32_t total = 0;
        if (tid < kBins) {
            const uint32_t d = tid;
            // prefix across waves (wave order = index order)
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) {
                const uint32_t c = s_wh[w][d];
                s_wh[w][d] = run;
                run += c;
            }
            total = run;
            // decoupled look-back: publish the aggregate, then walk back over
            // the predecessors LOOKBACK at a time until an inclusive prefix.
            // Statuses are partition-major (one 1-KB row per partition), so a
            // workgroup publishes into lines no other workgroup writes.
            uint32_t *col = status + d;
            uint32_t prefix = 0u;
            if (part == 0) {
                __hip_atomic_store(col, kFlagIncl | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(col + (size_t)part * kBins, kFlagAgg | total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                int64_t p = (int64_t)part - 1;
                while (true) {
                    uint32_t w[LOOKBACK];
#pragma unroll
                    for (int i = 0; i < LOOKBACK; ++i)
                        w[i] = (p - i >= 0) ? __hip_atomic_load(col + (size_t)(p - i) * kBins, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT)
                                            : kFlagIncl;  // never reached: partition 0 is inclusive
                    bool stop = false, incl = false;
                    int consumed = 0;
#pragma unroll
                    for (int i = 0; i < LOOKBACK; ++i) {
                        if (!stop) {
                            const uint32_t flag = w[i] & ~kCountMask;
                            if (flag == 0u) {
                                stop = true;  // not published yet: poll again from here
                            } else {
                                prefix += w[i] & kCountMask;
                                ++consumed;
                                if (flag == kFlagIncl) {
                                    incl = true;
                                    stop = true;
                                }
                            }
                        }
                    }
                    if (incl) break;
                    p -= consumed;
                    if (consumed < LOOKBACK) __builtin_amdgcn_s_sleep(1);
                }
                __hip_atomic_store(col + (size_t)part * kBins, kFlagIncl | (prefix + total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            s_glob[d] = s_base[d] + prefix;
            s_scan[d] = total;
        }
        __syncthreads();
        // block-local exclusive scan of the digit totals
        for (int off = 1; off < kBins; off <<= 1) {
            uint32_t t = 0u;
            if (tid < kBins && tid >= off) t = s_scan[tid - off];
            __syncthreads();
            if (tid < kBins) s_scan[tid] += t;
            __syncthreads();
        }
        if (tid < kBins) s_local[tid] = s_scan[tid] - total;
        if (tid == 0) s_next = atomicAdd(ticket, 1u);  // the next partition, taken ahead of the scatter
        __syncthreads();
        // stage into LDS in block-local sorted order
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            if (dig[j] != 0xFFFFFFFFu) {
                const uint32_t pos = s_local[dig[j]] + s_wh[wave][dig[j]] + rank[j];
                s_keys[pos] = key[j];
                s_vals[pos] = val[j];
            }
        }
        __syncthreads();
        // each digit's run leaves as one contiguous stretch
        const int64_t nvalid64 = K - start;
        const int nvalid = nvalid64 < kSortBlock * ITEMS ? (int)nvalid64 : kSortBlock * ITEMS;
        for (int q = tid; q < nvalid; q += kSortBlock) {
            const uint64_t kk = s_keys[q];
            const uint32_t dd = (uint32_t)(kk >> shift) & (kBins - 1);
            const uint32_t dst = s_glob[dd] + (uint32_t)q - s_local[dd];
            if ((int64_t)dst >= K) continue;  // only reachable with inconsistent digit counts
            keys_out[dst] = kk;
            vals_out[dst] = s_vals[q];
        }
        __syncthreads();  // LDS is reused by the next partition
        part = s_next;
        for (int k = tid; k < kSortWaves * kBins; k += kSortBlock) (&s_wh[0][0])[k] = 0u;
        __syncthreads();
    }
}

// inclusive scan over the 256 threads of a workgroup (four waves)
__device__ __forceinline__ uint32_t block256_inclusive_scan(uint32_t v, uint32_t *s_w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    if (lane == 63) s_w[wave] = v;
    __syncthreads();
    for (int k = 0; k < wave; ++k) v += s_w[k];
    __syncthreads();
    return v;
}

// Global start of every digit of every pass: digit counts are the prefix
// sums of the difference arrays (the sum of the partial rows), and the start
// of digit d is the exclusive prefix of the counts.  One workgroup per pass.
__global__ void __launch_bounds__(kBins) digit_base_kernel(const uint32_t *hist_part /*[kHistRows][stride]*/,
                                                           int stride, uint32_t *base /*[passes][256]*/) {
    __shared__ uint32_t s_w[kBins / 64];
    const int d = threadIdx.x;
    const uint32_t *h = hist_part + blockIdx.x * kHistStride;
    uint32_t v = 0u;
#pragma unroll
    for (int r = 0; r < kHistRows; ++r) v += h[(size_t)r * stride + d];
    const uint32_t count = block256_inclusive_scan(v, s_w);
    const uint32_t running = block256_inclusive_scan(count, s_w);
    base[blockIdx.x * kBins + d] = running - count;
}

// ---------------------------------------------------------------------------
// bucket sort by tile (the default when the tile count is moderate)
// ---------------------------------------------------------------------------
// The sorted order is (tile, depth bits, instance).  Instead of sorting all
// key bits across the whole array, keys are counted per (emission workgroup,
// tile), the counts are scanned into per-workgroup slots inside each tile's
// bucket, the keys are scattered there as (depth bits, instance) pairs, and
// each tile's bucket is sorted on its own in LDS.  The scatter order inside a
// bucket is arbitrary, but the pairs are distinct, so the per-tile sort
// alone fixes the order -- the same order a stable sort of (tile, depth)
// keys emitted in instance order produces.

// per tile t (one wave each): exclusive scan of the per-workgroup counts
// along the tile's row (in place) and the tile's total
__global__ void __launch_bounds__(256) bucket_colscan_kernel(uint32_t *cnt /*[n_tiles][rows]*/, int n_rows,
                                                             int64_t n_tiles, uint32_t *tile_count) {
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= n_tiles) return;  // uniform per wave
    uint32_t *row = cnt + (size_t)t * n_rows;
    uint32_t carry = 0u;
    for (int r0 = 0; r0 < n_rows; r0 += 256) {  // 4 consecutive counts per lane
        uint32_t c[4], sum = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = r0 + lane * 4 + k;
            c[k] = r < n_rows ? row[r] : 0u;
            sum += c[k];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        uint32_t run = carry + incl - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = r0 + lane * 4 + k;
            if (r < n_rows) row[r] = run;
            run += c[k];
        }
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) tile_count[t] = carry;
}

// ---------------------------------------------------------------------------
// tile work order (one workgroup of 1024 threads): a counting sort of each
// queue's items by descending list chunks
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t order_bin(uint32_t len) {
    const uint32_t chunks = len >> 6;
    return (uint32_t)(kOrderBins - 1) - (chunks < (uint32_t)(kOrderBins - 1) ? chunks : (uint32_t)(kOrderBins - 1));
}

// s_cnt[q][b] holds the item count of bin b of queue q; turns every row into
// its exclusive prefix (one wave per queue, one bin per lane)
__device__ __forceinline__ void order_bin_starts(uint32_t (*s_cnt)[kOrderBins]) {
    static_assert(kOrderBins == 64 && kOrderQueues <= 16, "one wave per queue, one lane per bin");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (wave < kOrderQueues) {
        const uint32_t c = s_cnt[wave][lane];
        uint32_t incl = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        s_cnt[wave][lane] = incl - c;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(1024) tile_order_kernel(const uint2 *ranges, int64_t n_items, uint32_t *order) {
    __shared__ uint32_t s_cnt[kOrderQueues][kOrderBins];
    const int tid = threadIdx.x;
    const int64_t qs = order_stride(n_items);
    for (int i = tid; i < kOrderQueues * kOrderBins; i += 1024) (&s_cnt[0][0])[i] = 0u;
    __syncthreads();
    for (int64_t t = tid; t < n_items; t += 1024) {
        const uint2 r = ranges[t];
        atomicAdd(&s_cnt[t % kOrderQueues][order_bin(r.y - r.x)], 1u);
    }
    order_bin_starts(s_cnt);
    for (int64_t t = tid; t < n_items; t += 1024) {
        const uint2 r = ranges[t];
        const int q = (int)(t % kOrderQueues);
        order[q * qs + atomicAdd(&s_cnt[q][order_bin(r.y - r.x)], 1u)] = (uint32_t)t;
    }
}

hipError_t launch_tile_order(const uint32_t *ranges, int64_t n_items, uint32_t *order, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    return launch_kernel(tile_order_kernel, dim3(1), dim3(1024), s, reinterpret_cast<const uint2 *>(ranges), n_items,
                         order);
}

// exclusive scan of the tile totals (one workgroup): the key count and the
// overflow flag (count above the capacity), each tile's first key, and the
// ranges ([first, end) for tiles with keys, [0, 0) otherwise, and all [0, 0)
// after an overflow)
__global__ void __launch_bounds__(1024) bucket_tilescan_kernel(const uint32_t *tile_count, int64_t n_tiles,
                                                               int64_t capacity, uint32_t *tile_start,
                                                               uint32_t *ranges, uint32_t *order, int64_t *d_num,
                                                               int32_t *d_overflow) {
    __shared__ uint64_t s_w[16];
    __shared__ uint32_t s_cnt[kOrderQueues][kOrderBins];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t per = (n_tiles + 1023) / 1024;
    const int64_t t0 = (int64_t)tid * per, t1 = (t0 + per < n_tiles) ? t0 + per : n_tiles;
    uint64_t sum = 0u;
    for (int64_t t = t0; t < t1; ++t) sum += tile_count[t];
    uint64_t incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t run = incl - sum, total = 0u;
    for (int k = 0; k < 16; ++k) {
        if (k < wave) run += s_w[k];
        total += s_w[k];
    }
    const bool ovf = total > (uint64_t)capacity;  // then every range is [0, 0)
    if (tid == 0) {
        *d_num = (int64_t)total;
        *d_overflow = ovf ? 1 : 0;
    }
    for (int64_t t = t0; t < t1; ++t) {
        const uint32_t c = tile_count[t];
        tile_start[t] = (uint32_t)run;
        ranges[2 * t] = (c && !ovf) ? (uint32_t)run : 0u;
        ranges[2 * t + 1] = (c && !ovf) ? (uint32_t)(run + c) : 0u;
        run += c;
    }
    if (!order) return;  // uniform
    // the work order of the lists just ranged (empty ones after an overflow)
    for (int i = tid; i < kOrderQueues * kOrderBins; i += 1024) (&s_cnt[0][0])[i] = 0u;
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) atomicAdd(&s_cnt[t % kOrderQueues][order_bin(ovf ? 0u : tile_count[t])], 1u);
    order_bin_starts(s_cnt);
    const int64_t qs = order_stride(n_tiles);
    for (int64_t t = t0; t < t1; ++t) {
        const int q = (int)(t % kOrderQueues);
        order[q * qs + atomicAdd(&s_cnt[q][order_bin(ovf ? 0u : tile_count[t])], 1u)] = (uint32_t)t;
    }
}

// Ascending bitonic sort in place in HBM of s[0, n2) (n2 a power of two) by
// a workgroup of THREADS threads, for buckets too long for LDS.  Each merge
// starts with the reflected compare (i, block end - 1 - i), so every
// compare-exchange is ascending and entries at or beyond `lim` act as
// +infinity without being stored; every step ends with a workgroup barrier.
__device__ __forceinline__ void compare_exchange_hbm(uint64_t *s, uint32_t i, uint32_t p, uint32_t lim) {
    if (p >= lim) return;
    const uint64_t a = s[i], b = s[p];
    const bool sw = a > b;
    s[i] = sw ? b : a;
    s[p] = sw ? a : b;
}

template <int THREADS>
__device__ __forceinline__ void bitonic_sort_hbm(uint64_t *s, uint32_t n2, uint32_t lim) {
    const uint32_t tid = threadIdx.x, half = n2 >> 1;
    for (uint32_t lk = 1; (1u << lk) <= n2; ++lk) {
        const uint32_t k = 1u << lk;
        {
            const uint32_t lj = lk - 1, j = k >> 1;
            for (uint32_t t = tid; t < half; t += THREADS) {
                const uint32_t base = (t >> lj) << lk, r = t & (j - 1);
                compare_exchange_hbm(s, base + r, base + (k - 1 - r), lim);
            }
            __syncthreads();
        }
        for (int lj = (int)lk - 2; lj >= 0; --lj) {
            const uint32_t j = 1u << lj;
            for (uint32_t t = tid; t < half; t += THREADS) {
                const uint32_t i = ((t >> lj) << (lj + 1)) + (t & (j - 1));
                compare_exchange_hbm(s, i, i + j, lim);
            }
            __syncthreads();
        }
    }
}

// Bitonic sort of a bucket in LDS with E = 2^P entries per thread and up to
// P network steps per LDS round trip.  A group is the E positions
// base + m * 2^lo (m < E, mask bits lo .. lo+P-1); one pass loads a group
// into registers, applies the compare-exchanges of the top `b` mask bits (the
// network's next steps), and stores it back.  Merge k = 2^lk runs its steps
// bit lk-1 down to bit P in passes of up to P bits, then bits P-1 .. 0 in one
// pass over E consecutive positions; merges up to E happen in registers
// right after the bucket is read.  The network is the classic one (merge lk
// sorts descending where bit lk of the position is set, except the final
// merge); instead of a direction per compare-exchange, an entry is held
// bit-complemented while its merge runs descending, so every compare-exchange
// is ascending, and entries are complemented or restored only where one
// merge hands over to the next.  LDS slot i + i / E keeps the strided passes
// free of bank conflicts.  With several waves on one bucket, a pass whose mask
// stays below bit 6 + P only touches the 64 E positions its wave owns (higher
// position bits come from the wave index), so two such passes in a row need
// no workgroup barrier; a bucket sorted by one wave never needs one.
template <int P>
__device__ __forceinline__ uint32_t lds_slot(uint32_t i) {
    return i + (i >> P);
}

__device__ __forceinline__ void cmp_swap_up(uint64_t &a, uint64_t &b) {
    const bool sw = a > b;
    const uint64_t lo = sw ? b : a, hi = sw ? a : b;
    a = lo;
    b = hi;
}

// ascending compare-exchanges along mask bits r = P-1 .. P-B of the group
template <int P, int B>
__device__ __forceinline__ void group_steps(uint64_t (&v)[1 << P]) {
#pragma unroll
    for (int r = P - 1; r > P - 1 - B; --r) {
#pragma unroll
        for (int m = 0; m < (1 << P); ++m)
            if (!(m & (1 << r))) cmp_swap_up(v[m], v[m | (1 << r)]);
    }
}

__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// all-ones when the entry at a position with bit `j` equal to `bit` is held
// complemented during merge j of a network of 2^ln entries
__device__ __forceinline__ uint64_t held_mask(int j, int ln, uint32_t bit) {
    return (j < ln && bit) ? ~0ull : 0ull;
}

// Sorts the L entries at in[0, L) (n2 = 2^ln >= max(L, 2^P); s holds at
// least lds_slot<P>(n2) entries) with NT threads (tid < NT; NT = 64 and
// ONE_WAVE for a wave on its own) and writes key (thi | depth bits) and value
// (instance) of sorted entry p to keys[p], vals[p].
template <int NT, int P, bool ONE_WAVE>
__device__ __forceinline__ void sort_bucket_lds(uint64_t *s, const uint64_t *in, uint32_t L, uint32_t n2, int ln,
                                                uint64_t thi, uint64_t *keys, uint32_t *vals, uint32_t tid) {
    constexpr int E = 1 << P;
    const uint32_t groups = n2 >> P;
    // merges of 2 .. E in registers.  Input j = m * groups + g takes
    // position E g + m (any placement is valid; this one reads coalesced).
    for (uint32_t g = tid; g < groups; g += NT) {
        uint64_t v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const uint32_t j = (uint32_t)m * groups + g;
            v[m] = j < L ? in[j] : ~0ull;
        }
#pragma unroll
        for (int lk = 1; lk <= P; ++lk) {
            // hand over from merge lk-1 to merge lk (bit P of the position is bit 0 of g)
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const uint32_t cur = lk < P ? ((m >> lk) & 1) : (g & 1u);
                const uint32_t prev = (m >> (lk - 1)) & 1;
                v[m] ^= held_mask(lk, ln, cur) ^ (lk > 1 ? held_mask(lk - 1, ln, prev) : 0ull);
            }
#pragma unroll
            for (int lj = lk - 1; lj >= 0; --lj)
#pragma unroll
                for (int m = 0; m < E; ++m)
                    if (!(m & (1 << lj))) cmp_swap_up(v[m], v[m | (1 << lj)]);
        }
        const uint32_t base = g << P;
        if (ln == P) {  // merge P was the final one: nothing is held complemented
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (base + m < L) {
                    keys[base + m] = thi | (v[m] >> 32);
                    vals[base + m] = (uint32_t)v[m];
                }
        } else {
            const uint64_t flip = held_mask(P, ln, g & 1u) ^ held_mask(P + 1, ln, (g >> 1) & 1u);
#pragma unroll
            for (int m = 0; m < E; ++m) s[lds_slot<P>(base + m)] = v[m] ^ flip;
        }
    }
    int top_prev = P - 1;
    for (int lk = P + 1; lk <= ln; ++lk) {
        const bool fin = lk == ln;
        for (int hi = lk - 1;;) {
            // mask bits hi-P+1 .. hi; compare-exchanges along the top b of them
            const bool low = hi == P - 1;
            const int b = low ? P : (hi - (P - 1) < P ? hi - (P - 1) : P), lo = hi - (P - 1);
            if (!ONE_WAVE && (hi >= 6 + P || top_prev >= 6 + P))
                __syncthreads();
            else
                lds_wave_sync();
            top_prev = hi;
            for (uint32_t g = tid; g < groups; g += NT) {
                const uint32_t base = ((g >> lo) << (lo + P)) | (g & ((1u << lo) - 1u));
                uint64_t v[E];
#pragma unroll
                for (int m = 0; m < E; ++m) v[m] = s[lds_slot<P>(base + ((uint32_t)m << lo))];
                if (b == P)
                    group_steps<P, P>(v);
                else if (b == 1)
                    group_steps<P, 1>(v);
                else if (b == 2)
                    group_steps<P, (P > 2 ? 2 : 1)>(v);
                else
                    group_steps<P, (P > 3 ? 3 : 1)>(v);
                if (fin && low) {  // E consecutive sorted entries, none held complemented
#pragma unroll
                    for (int m = 0; m < E; ++m)
                        if (base + m < L) {
                            keys[base + m] = thi | (v[m] >> 32);
                            vals[base + m] = (uint32_t)v[m];
                        }
                } else {
                    // the last pass of a merge hands over to the next merge
                    const uint64_t flip = low ? held_mask(lk, ln, (base >> lk) & 1u) ^
                                                    held_mask(lk + 1, ln, (base >> (lk + 1)) & 1u)
                                              : 0ull;
#pragma unroll
                    for (int m = 0; m < E; ++m) s[lds_slot<P>(base + ((uint32_t)m << lo))] = v[m] ^ flip;
                }
            }
            if (low) break;
            hi -= b;
        }
    }
}

// Buckets of up to kSmallSortCap entries: a 256-thread workgroup each (up
// to seven resident per CU); longer ones: a 512-thread workgroup each, in LDS
// up to kTileSortCap, in place in HBM beyond.  Eight entries per thread.
constexpr int kSmallSortBlock = 256, kSmallSortCap = 2048;
constexpr int kTileSortBlock = 512, kTileSortCap = 8192;

// One workgroup per tile (grid-stride): sort the bucket and write the keys
// (tile << 32 | depth bits) and values (instance).  Launched twice: small
// workgroups for buckets of 1..kSmallSortCap entries, then large ones for the
// rest.
template <int THREADS, int CAP, bool SMALL>
__global__ void __launch_bounds__(THREADS) tile_sort_kernel(uint64_t *bucket, const uint32_t *ranges,
                                                            int64_t n_tiles, int64_t n_blocks, uint64_t *keys,
                                                            uint32_t *vals, const int32_t *d_overflow) {
    __shared__ uint64_t s[CAP + CAP / 8];
    if (*d_overflow) return;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += n_blocks) {  // uniform per workgroup
        const uint32_t b = ranges[2 * tile], L = ranges[2 * tile + 1] - b;
        if (L == 0u || (SMALL ? L > (uint32_t)kSmallSortCap : L <= (uint32_t)kSmallSortCap)) continue;
        uint32_t n2 = 8;
        int ln = 3;
        while (n2 < L) n2 <<= 1, ++ln;
        const uint64_t thi = (uint64_t)tile << 32;
        if (L <= (uint32_t)CAP) {
            sort_bucket_lds<THREADS, 3, false>(s, bucket + b, L, n2, ln, thi, keys + b, vals + b, threadIdx.x);
        } else {
            bitonic_sort_hbm<THREADS>(bucket + b, n2, L);
            for (uint32_t i = threadIdx.x; i < L; i += THREADS) {
                const uint64_t c = bucket[b + i];
                keys[b + i] = thi | (c >> 32);
                vals[b + i] = (uint32_t)c;
            }
        }
        __syncthreads();  // s and the bucket are reused by the next tile
    }
}

// ---------------------------------------------------------------------------
// tile ranges
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) ranges_kernel(const uint64_t *keys, const int64_t *d_num, int64_t capacity,
                                                     const int32_t *d_overflow, uint32_t *ranges,
                                                     uint64_t n_tiles_total, int64_t stride) {
    if (*d_overflow) return;
    const int64_t K = sort_count(d_num, capacity);
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < K; k += stride) {
        const uint64_t t = keys[k] >> 32;
        if (t >= n_tiles_total) continue;
        if (k == 0 || (keys[k - 1] >> 32) != t) ranges[2 * t] = (uint32_t)k;
        if (k == K - 1 || (keys[k + 1] >> 32) != t) ranges[2 * t + 1] = (uint32_t)(k + 1);
    }
}

// ---------------------------------------------------------------------------
// host side of the pipeline
// ---------------------------------------------------------------------------


static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SortPlan make_sort_plan(int64_t n, int64_t capacity, int64_t n_tiles_total) {
    SortPlan p;
    p.part_keys = kMinSortPart;
    p.lookback = 16;
    p.n = n;
    p.capacity = capacity;
    p.n_tiles_total = n_tiles_total;
    int tb = 1;
    while ((1ll << tb) < n_tiles_total) ++tb;
    p.tile_bits = tb;
    p.passes = (32 + tb + kRadixBits - 1) / kRadixBits;
    p.scan_blocks = (n + kScanTile - 1) / kScanTile;
    if (p.scan_blocks < 1) p.scan_blocks = 1;
    p.sort_parts = (capacity + kMinSortPart - 1) / kMinSortPart;
    if (p.sort_parts < 1) p.sort_parts = 1;
    size_t o = 0;
    p.off_part = o;
    o = align256(o + sizeof(uint64_t) * (size_t)p.scan_blocks);
    p.off_keys2 = o;
    o = align256(o + sizeof(uint64_t) * (size_t)(capacity > 0 ? capacity : 1));
    p.off_vals2 = o;
    o = align256(o + sizeof(uint32_t) * (size_t)(capacity > 0 ? capacity : 1));
    p.off_rows = o;
    o = align256(o + sizeof(uint32_t) * (size_t)kEmitGrid * p.passes * kHistStride);
    p.off_dbase = o;
    o = align256(o + sizeof(uint32_t) * (size_t)kMaxPasses * kBins);
    // histogram partials, status and tickets are contiguous so one fill clears them
    p.off_hist = o;
    o = o + sizeof(uint32_t) * (size_t)kHistRows * kMaxPasses * kHistStride;
    p.off_ticket = o;
    o = o + sizeof(uint32_t) * (size_t)kMaxPasses * 64;
    p.off_status = o;
    o = o + sizeof(uint32_t) * (size_t)p.passes * (size_t)p.sort_parts * kBins;
    o = align256(o);
    // bucket path (moderate tile counts): per-workgroup tile counters, tile totals and starts
    p.bucket_ok = n_tiles_total <= kBucketMaxTiles;
    p.bucket_blocks = p.scan_blocks < kBucketGrid ? p.scan_blocks : kBucketGrid;
    p.off_tcnt = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)p.bucket_blocks * (size_t)n_tiles_total);
    p.off_tcount = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)n_tiles_total);
    p.off_tstart = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)n_tiles_total);
    p.use_bucket = p.bucket_ok;
    p.total = align256(o);
    return p;
}

// the bucket path after the scan: count per (workgroup, tile), scan the
// counters, scatter into the buckets, sort each bucket
static hipError_t run_bucket_sort(const SortPlan &P, const uint32_t *tt, const float4 *rec, int TX, int TY,
                                  char *ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges, uint32_t *order,
                                  int64_t *d_num, int32_t *d_overflow, int n_cu, hipStream_t s) {
    hipError_t e;
    if (P.n <= 0) {  // no keys: count 0, no overflow, every range empty
        if ((e = launch_kernel(scan_partials_kernel, dim3(1), dim3(1024), s, (uint64_t *)nullptr, (int64_t)0,
                               P.capacity, d_num, d_overflow)) != hipSuccess)
            return e;
        if ((e = launch_fill_u32(ranges, 0u, 2 * P.n_tiles_total, s)) != hipSuccess) return e;
        return order ? launch_tile_order(ranges, P.n_tiles_total, order, s) : hipSuccess;
    }
    EmitArgs A = {};
    A.tt = tt;
    A.rec = rec;
    A.n = P.n;
    A.n_tiles_scan = P.scan_blocks;
    A.capacity = P.capacity;
    A.n_blocks = P.bucket_blocks;
    A.TX = TX;
    A.TY = TY;
    A.tile_cnt = reinterpret_cast<uint32_t *>(ws + P.off_tcnt);
    A.tile_start = reinterpret_cast<const uint32_t *>(ws + P.off_tstart);
    A.bucket = reinterpret_cast<uint64_t *>(ws + P.off_keys2);
    A.n_tiles = P.n_tiles_total;
    A.d_overflow = d_overflow;
    uint32_t *tcount = reinterpret_cast<uint32_t *>(ws + P.off_tcount);
    uint32_t *tstart = reinterpret_cast<uint32_t *>(ws + P.off_tstart);
    if ((e = launch_kernel(emit_kernel<kEmitCountTiles>, dim3((unsigned)P.bucket_blocks), dim3(kEmitBlock), s, A)) !=
        hipSuccess)
        return e;
    if ((e = launch_kernel(bucket_colscan_kernel, dim3((unsigned)((P.n_tiles_total + 3) / 4)), dim3(256), s,
                           A.tile_cnt, (int)P.bucket_blocks, P.n_tiles_total, tcount)) != hipSuccess)
        return e;
    if ((e = launch_kernel(bucket_tilescan_kernel, dim3(1), dim3(1024), s, (const uint32_t *)tcount, P.n_tiles_total,
                           P.capacity, tstart, ranges, order, d_num, d_overflow)) != hipSuccess)
        return e;
    if ((e = launch_kernel(emit_kernel<kEmitScatterTiles>, dim3((unsigned)P.bucket_blocks), dim3(kEmitBlock), s,
                           A)) != hipSuccess)
        return e;
    int64_t sg = 8 * (int64_t)n_cu;
    if (sg > P.n_tiles_total) sg = P.n_tiles_total;
    if ((e = launch_kernel(tile_sort_kernel<kSmallSortBlock, kSmallSortCap, true>, dim3((unsigned)sg),
                           dim3(kSmallSortBlock), s, A.bucket, (const uint32_t *)ranges, P.n_tiles_total, sg, keys,
                           vals, d_overflow)) != hipSuccess)
        return e;
    int64_t lg = (int64_t)n_cu;
    if (lg > P.n_tiles_total) lg = P.n_tiles_total;
    return launch_kernel(tile_sort_kernel<kTileSortBlock, kTileSortCap, false>, dim3((unsigned)lg),
                         dim3(kTileSortBlock), s, A.bucket, (const uint32_t *)ranges, P.n_tiles_total, lg, keys, vals,
                         d_overflow);
}

hipError_t run_bin_sort(const SortPlan &P, const uint32_t *tt, const float4 *rec, int TX, int TY, char *ws,
                        uint64_t *keys, uint32_t *vals, uint32_t *ranges, uint32_t *order, int64_t *d_num,
                        int32_t *d_overflow, int n_cu, hipStream_t s) {
    hipError_t e;
    uint64_t *part = reinterpret_cast<uint64_t *>(ws + P.off_part);
    uint64_t *keys2 = reinterpret_cast<uint64_t *>(ws + P.off_keys2);
    uint32_t *vals2 = reinterpret_cast<uint32_t *>(ws + P.off_vals2);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + P.off_hist);
    uint32_t *rows = reinterpret_cast<uint32_t *>(ws + P.off_rows);
    uint32_t *dbase = reinterpret_cast<uint32_t *>(ws + P.off_dbase);
    uint32_t *ticket = reinterpret_cast<uint32_t *>(ws + P.off_ticket);
    uint32_t *status = reinterpret_cast<uint32_t *>(ws + P.off_status);
    const size_t clear_words = (P.off_status - P.off_hist) / 4 + (size_t)P.passes * P.sort_parts * kBins;

    // clears the onesweep state and the ranges; the bucket path writes every
    // counter and every range itself
    if (!P.use_bucket) {
        if ((e = launch_kernel(clear2_kernel, dim3(1024), dim3(256), s, hist, (int64_t)clear_words, ranges,
                               2 * P.n_tiles_total, (int64_t)1024 * 256)) != hipSuccess)
            return e;
    }
    // the bucket path counts keys per tile and needs no scan over instances
    if (P.use_bucket)
        return run_bucket_sort(P, tt, rec, TX, TY, ws, keys, vals, ranges, order, d_num, d_overflow, n_cu, s);
    // 1. scan
    if (P.n > 0) {
        if ((e = launch_kernel(scan_reduce_kernel, dim3((unsigned)P.scan_blocks), dim3(kScanBlock), s, tt, P.n,
                               part)) != hipSuccess)
            return e;
    }
    if ((e = launch_kernel(scan_partials_kernel, dim3(1), dim3(1024), s, part, P.n > 0 ? P.scan_blocks : (int64_t)0,
                           P.capacity, d_num, d_overflow)) != hipSuccess)
        return e;
    // 2. emission (with the scan downsweep) into the buffer that the last pass does not write to
    const bool odd = (P.passes & 1) != 0;
    uint64_t *k_a = odd ? keys2 : keys;
    uint32_t *v_a = odd ? vals2 : vals;
    uint64_t *k_b = odd ? keys : keys2;
    uint32_t *v_b = odd ? vals : vals2;
    if (P.n > 0) {
        int64_t eg = P.scan_blocks;
        if (eg > kEmitGrid) eg = kEmitGrid;
        EmitArgs A = {};
        A.tt = tt;
        A.part = part;
        A.rec = rec;
        A.n = P.n;
        A.n_tiles_scan = P.scan_blocks;
        A.capacity = P.capacity;
        A.n_blocks = eg;
        A.TX = TX;
        A.TY = TY;
        A.keys = k_a;
        A.vals = v_a;
        A.passes = P.passes;
        A.rows = rows;
        A.d_overflow = d_overflow;
        if ((e = launch_kernel(emit_kernel<kEmitSortKeys>, dim3((unsigned)eg), dim3(kEmitBlock), s, A)) != hipSuccess)
            return e;
        const int cols = P.passes * kHistStride;
        if ((e = launch_kernel(hist_reduce_kernel, dim3((unsigned)((cols + 63) / 64), kHistRows), dim3(256), s, rows,
                               (int)eg, cols, hist)) != hipSuccess)
            return e;
        if ((e = launch_kernel(digit_base_kernel, dim3((unsigned)P.passes), dim3(kBins), s, hist, cols, dbase)) !=
            hipSuccess)
            return e;
    }
    // 3. onesweep passes over the significant bits (digit counts come from the emission)
    // persistent grid: one workgroup per CU (60 or 110 KB of LDS)
    using SweepFn = void (*)(const uint64_t *, const uint32_t *, uint64_t *, uint32_t *, const int64_t *, int64_t,
                             int, const uint32_t *, uint32_t *, uint32_t *, const int32_t *);
    SweepFn sweep;
    const int part_keys = (P.part_keys == 2 * kMinSortPart) ? 2 * kMinSortPart : kMinSortPart;
    if (part_keys == kMinSortPart)
        sweep = P.lookback >= 64 ? onesweep_kernel<8, 64> : P.lookback >= 32 ? onesweep_kernel<8, 32>
                                                                              : onesweep_kernel<8, 16>;
    else
        sweep = P.lookback >= 64 ? onesweep_kernel<16, 64> : P.lookback >= 32 ? onesweep_kernel<16, 32>
                                                                               : onesweep_kernel<16, 16>;
    // two persistent workgroups per CU (the LDS of each allows two): while
    // one waits on its look-back or loads, the other ranks or scatters
    int64_t sg = 2 * (int64_t)n_cu;
    const int64_t parts_used = (P.capacity + part_keys - 1) / part_keys;
    if (sg > parts_used) sg = parts_used;
    if (sg < 1) sg = 1;
    for (int p = 0; p < P.passes; ++p) {
        if ((e = launch_kernel(sweep, dim3((unsigned)sg), dim3(kSortBlock), s, k_a, v_a, k_b, v_b, d_num,
                               P.capacity, p * kRadixBits, dbase + p * kBins,
                               status + (size_t)p * P.sort_parts * kBins, ticket + p * 64, d_overflow)) != hipSuccess)
            return e;
        uint64_t *tk = k_a;
        k_a = k_b;
        k_b = tk;
        uint32_t *tv = v_a;
        v_a = v_b;
        v_b = tv;
    }
    // k_a now holds the sorted keys (== keys)
    // 4. ranges
    {
        int64_t blocks = (P.capacity + 255) / 256;
        if (blocks > (int64_t)n_cu * 4) blocks = (int64_t)n_cu * 4;
        if ((e = launch_kernel(ranges_kernel, dim3((unsigned)blocks), dim3(256), s, k_a, d_num, P.capacity,
                               d_overflow, ranges, (uint64_t)P.n_tiles_total, blocks * 256)) != hipSuccess)
            return e;
    }
    // 5. the compositing work order
    return order ? launch_tile_order(ranges, P.n_tiles_total, order, s) : hipSuccess;
}

}  // namespace gs
