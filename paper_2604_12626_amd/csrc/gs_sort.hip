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
constexpr int kWinGrid = 1024;    // the same with windowed counters (each a contiguous run of scan tiles)
constexpr int64_t kBucketMaxTiles = 4096;  // tile counters in LDS up to this many tiles (all views)
constexpr int64_t kWindowMaxTiles = 1 << 18;  // beyond: windowed counters, up to this many (a 256 MB table)
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

enum EmitMode { kEmitSortKeys = 0, kEmitCountTiles = 1, kEmitScatterTiles = 2, kEmitCountWin = 3, kEmitScatterWin = 4 };

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
    // kEmitCountWin / kEmitScatterWin (more tiles than LDS holds): each
    // workgroup takes a contiguous run of scan tiles and counts in an LDS
    // window of win_views whole views (T tiles each), a ring that moves
    // forward with the views; a tile's count leaves the window once, with
    // its view, by one atomic on tile_count that returns the workgroup's
    // offset inside the tile's windowed keys (kept in tile_cnt, here
    // [grid][n_tiles]); keys of views beyond the window (a block drawing
    // more views than it holds) count on tile_over
    uint32_t *tile_count;  // [n_tiles]: windowed keys per tile
    uint32_t *tile_over;   // [n_tiles]: keys counted outside a window (count up, scatter down to 0)
    int64_t T;             // tiles per view
    int win_views;         // views per window (kLdsTiles / T)
    // count modes write, scatter modes read, the live instances of every
    // (scan tile, wave): comp[(tile * kEmitWaves + wave) * kWaveInst + e] =
    // {first tile, rect width | height << 16, depth bits, instance}, and
    // their number in comp_n[tile * kEmitWaves + wave]
    uint4 *comp;
    uint32_t *comp_n;
};

template <int MODE>
__global__ void __launch_bounds__(kEmitBlock) emit_kernel(const EmitArgs A) {
    // digit histograms (sort keys) or, for up to kLdsTiles tiles, the
    // workgroup's tile counters (count / scatter)
    __shared__ uint32_t s_aux[kLdsTiles];
    uint32_t(*s_h)[kHistStride] = reinterpret_cast<uint32_t(*)[kHistStride]>(s_aux);
    __shared__ uint64_t s_wsum[kEmitWaves];
    // per wave, per list entry: staged record, then the emission layout
    __shared__ uint32_t s_a0[kEmitWaves][kWaveInst];  // u bits          -> first tile of the rect
    __shared__ uint32_t s_a1[kEmitWaves][kWaveInst];  // v bits          -> rect width
    __shared__ uint32_t s_a2[kEmitWaves][kWaveInst];  // depth bits
    __shared__ uint32_t s_a3[kEmitWaves][kWaveInst];  // radius
    __shared__ uint32_t s_a4[kEmitWaves][kWaveInst];  // view
    __shared__ uint32_t s_a5[kEmitWaves][kWaveInst];  // instance index
    __shared__ uint32_t s_a6[kEmitWaves][kWaveInst];  // first key, relative to the wave's first
    __shared__ uint32_t s_a7[kEmitWaves][kWaveInst];  // tiles_touched
    // per wave: the lanes of a 64-key window where a list entry starts (tagged
    // with the window's number, so no clearing between windows)
    __shared__ uint32_t s_flag[kEmitWaves][64];
    if ((MODE == kEmitScatterTiles || MODE == kEmitScatterWin) && *A.d_overflow) return;  // nothing consistent to scatter
    const uint32_t *tt = A.tt;
    const float4 *rec = A.rec;
    const int64_t n = A.n, capacity = A.capacity;
    const int TX = A.TX, TY = A.TY, passes = A.passes;
    if (MODE == kEmitSortKeys)
        for (int k = threadIdx.x; k < kMaxPasses * kHistStride; k += kEmitBlock) s_aux[k] = 0u;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    s_flag[wave][lane] = 0u;
    uint32_t tag = 0u;  // windows this wave has walked
    // tile counters in HBM are tile-major: tile t's counts of all workgroups are one row
    uint32_t *my_cnt = A.tile_cnt + blockIdx.x;
    const int64_t cs = A.n_blocks;  // row stride
    // count / scatter: the tile counters live in LDS (at most kLdsTiles tiles)
    if (MODE == kEmitCountTiles)
        for (int k = threadIdx.x; k < A.n_tiles; k += kEmitBlock) s_aux[k] = 0u;
    if (MODE == kEmitScatterTiles)  // this workgroup's first slot in every bucket
        for (int k = threadIdx.x; k < A.n_tiles; k += kEmitBlock) s_aux[k] = A.tile_start[k] + my_cnt[k * cs];
    if (MODE == kEmitCountTiles || MODE == kEmitScatterTiles) __syncthreads();  // the counters are set
    constexpr bool WIN = MODE == kEmitCountWin || MODE == kEmitScatterWin;
    // per wave, the views of its block (two blocks' worth: a wave may be one
    // block ahead of the others, up to the next window barrier)
    __shared__ uint32_t s_vmin[2][kEmitWaves], s_vmax[2][kEmitWaves];
    // window [win_base, win_base + win_tiles) of global tiles (uniform)
    const uint32_t win_tiles = WIN ? (uint32_t)(A.win_views * A.T) : 0u;
    // the windowed offsets are workgroup-major: a window's are contiguous
    uint32_t *my_row = A.tile_cnt + (WIN ? (size_t)blockIdx.x * (size_t)A.n_tiles : 0u);
    int64_t win_lo = -1;  // first view of the window, -1 before the first
    uint32_t win_base = 0u, ring_off = 0u;  // first tile of the window, its place in the ring
    if (MODE == kEmitCountWin)
        for (int k = threadIdx.x; k < kLdsTiles; k += kEmitBlock) s_aux[k] = 0u;
    // windowed modes: a contiguous run of scan tiles per workgroup, so its
    // instances -- and their views -- come in increasing order
    const int64_t t_first = WIN ? (int64_t)blockIdx.x * A.n_tiles_scan / A.n_blocks : (int64_t)blockIdx.x;
    const int64_t t_last = WIN ? ((int64_t)blockIdx.x + 1) * A.n_tiles_scan / A.n_blocks : A.n_tiles_scan;
    const int64_t t_step = WIN ? 1 : A.n_blocks;
    // the ring slots of views [v0, v1) (v1 - v0 <= win_views): count mode
    // hands their counts to the tiles (one atomic per nonzero tile returns
    // this workgroup's offset in the tile) and clears them; scatter mode
    // loads the workgroup's first slot in each of their tiles
    auto window_views = [&](int64_t v0, int64_t v1) {
        const uint32_t Tn = (uint32_t)A.T, m = (uint32_t)(v1 - v0) * Tn;
        for (uint32_t k = threadIdx.x; k < m; k += kEmitBlock) {
            const int64_t u = v0 + k / Tn;
            const uint32_t loc = k % Tn, slot = (uint32_t)(u % A.win_views) * Tn + loc;
            const uint64_t t = (uint64_t)u * Tn + loc;
            if (MODE == kEmitCountWin) {
                const uint32_t c = s_aux[slot];
                if (c && t < (uint64_t)A.n_tiles) my_row[t] = atomicAdd(A.tile_count + t, c);
                s_aux[slot] = 0u;
            } else {
                s_aux[slot] = t < (uint64_t)A.n_tiles ? A.tile_start[t] + my_row[t] : 0u;
            }
        }
    };
    static_assert(kEmitItems == 4, "one 16-B tiles_touched load per thread");
    // the thread's four tiles_touched of a scan tile: one 16-B load (tt is
    // 16-B aligned: caller-owned allocation), element-wise at the end
    auto load_tt = [&](int64_t tile) {
        const int64_t b = tile * kScanTile + (int64_t)threadIdx.x * kEmitItems;
        if (b + kEmitItems <= n) return *reinterpret_cast<const uint4 *>(tt + b);
        return make_uint4(b < n ? tt[b] : 0u, b + 1 < n ? tt[b + 1] : 0u, b + 2 < n ? tt[b + 2] : 0u,
                          b + 3 < n ? tt[b + 3] : 0u);
    };
    constexpr bool SCATTER = MODE == kEmitScatterTiles || MODE == kEmitScatterWin;
    constexpr bool COUNT = MODE == kEmitCountTiles || MODE == kEmitCountWin;
    // scatter modes read what the count pass kept instead of tiles_touched
    // and the records; the next block's counts are in flight meanwhile
    // The other modes keep two blocks in flight: at the start of a block the
    // records of the next one and the counts of the one after are requested.
    // The first 16 B of a record (u, v, depth, radius) are requested for
    // every instance of the lane, a culled one's replaced by the first record
    // (any record in bounds; never used), so that no request depends on a
    // branch.  Views increase with the instance, so the views of the wave's
    // first and last drawn instances bound them all: when they are equal,
    // no other view is read.
    auto load_rec = [&](const uint4 &qq, int64_t tile, float4 (&o)[kEmitItems], uint32_t &vf, uint32_t &vl) {
        const int64_t b = tile * kScanTile + (int64_t)threadIdx.x * kEmitItems;
        const uint32_t c[kEmitItems] = {qq.x, qq.y, qq.z, qq.w};
#pragma unroll
        for (int k = 0; k < kEmitItems; ++k) o[k] = rec[3 * (c[k] ? b + k : 0)];
        const uint64_t m = __ballot((c[0] | c[1] | c[2] | c[3]) != 0u);
        vf = vl = 0u;
        if (m) {  // uniform
            const int lf = __ffsll((unsigned long long)m) - 1, ll = 63 - __clzll((long long)m);
            const uint32_t kf = c[0] ? 0u : c[1] ? 1u : c[2] ? 2u : 3u, kl = c[3] ? 3u : c[2] ? 2u : c[1] ? 1u : 0u;
            const int64_t wb = tile * kScanTile + (int64_t)wave * kWaveInst;
            const int64_t i_f = wb + lf * kEmitItems + (int64_t)__builtin_amdgcn_readlane(kf, lf);
            const int64_t i_l = wb + ll * kEmitItems + (int64_t)__builtin_amdgcn_readlane(kl, ll);
            vf = (uint32_t)__float_as_int(rec[3 * i_f + 2].w);
            vl = (uint32_t)__float_as_int(rec[3 * i_l + 2].w);
        }
    };
    uint4 q_next = make_uint4(0u, 0u, 0u, 0u), q_next2 = make_uint4(0u, 0u, 0u, 0u);
    float4 qn[kEmitItems];
    uint32_t vfn = 0u, vln = 0u;
    uint32_t cn_next = 0u;
    if (t_first < t_last) {
        if (SCATTER) {
            cn_next = A.comp_n[t_first * kEmitWaves + wave];
        } else {
            q_next = load_tt(t_first);
            if (t_first + t_step < t_last) q_next2 = load_tt(t_first + t_step);
            load_rec(q_next, t_first, qn, vfn, vln);
        }
    }
    int par = 0;  // block parity
    for (int64_t tile = t_first; tile < t_last; tile += t_step, par ^= 1) {  // uniform per workgroup
        const int64_t cbase = (tile * kEmitWaves + wave) * kWaveInst;
        uint32_t wave_total = 0u, n_live = 0u;
        int64_t kw = 0, room = INT64_MAX;
        if (SCATTER) {
            n_live = cn_next;
            if (tile + t_step < t_last) cn_next = A.comp_n[(tile + t_step) * kEmitWaves + wave];
            uint4 r[kWaveInst / 64];
#pragma unroll
            for (int k = 0; k < kWaveInst / 64; ++k) {
                const uint32_t e = (uint32_t)(k * 64 + lane);
                r[k] = e < n_live ? A.comp[cbase + e] : make_uint4(0u, 0u, 0u, 0u);
            }
            // list starts: the exclusive scan of the rect sizes
#pragma unroll
            for (int k = 0; k < kWaveInst / 64; ++k) {
                const uint32_t e = (uint32_t)(k * 64 + lane);
                const uint32_t w = r[k].y & 0xFFFFu, c = w * (r[k].y >> 16);
                uint32_t incl = c;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint32_t y = __shfl_up(incl, off, 64);
                    if (lane >= off) incl += y;
                }
                if (e < n_live) {
                    s_a0[wave][e] = r[k].x;
                    s_a1[wave][e] = w;
                    s_a2[wave][e] = r[k].z;
                    s_a5[wave][e] = r[k].w;
                    s_a6[wave][e] = wave_total + incl - c;
                }
                wave_total += __shfl(incl, 63, 64);
            }
            __builtin_amdgcn_wave_barrier();
        } else {
            const int64_t base = tile * kScanTile + (int64_t)threadIdx.x * kEmitItems;
            // this block's counts and records; the next blocks' in flight meanwhile
            const uint4 q = q_next;
            float4 q0[kEmitItems];
#pragma unroll
            for (int k = 0; k < kEmitItems; ++k) q0[k] = qn[k];
            const uint32_t vf = vfn, vl = vln;
            q_next = q_next2;
            if (tile + 2 * t_step < t_last) q_next2 = load_tt(tile + 2 * t_step);
            if (tile + t_step < t_last) load_rec(q_next, tile + t_step, qn, vfn, vln);
            uint32_t v[kEmitItems] = {q.x, q.y, q.z, q.w};
            // wave-level inclusive scan of the per-thread sums (fits 32 bits:
            // 256 instances of at most 2^22 tiles), then across the waves in 64 bits
            uint32_t incl = v[0] + v[1] + v[2] + v[3];
            const uint32_t own = incl;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            wave_total = __shfl(incl, 63, 64);
            // sort keys go to the wave's stretch of the key array (first key kw,
            // nothing past the capacity); the bucket modes place keys by tile
            // counters instead and scatter only when the total fits
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
            n_live = __shfl(pos, 63, 64);
            pos -= cnt;
            // the views: one for the whole wave, or (at a view boundary) read
            uint32_t view[kEmitItems];
#pragma unroll
            for (int k = 0; k < kEmitItems; ++k) view[k] = vf;
            if (vf != vl) {  // uniform
#pragma unroll
                for (int k = 0; k < kEmitItems; ++k)
                    if (live_mask & (1u << k)) view[k] = (uint32_t)__float_as_int(rec[3 * (base + k) + 2].w);
            }
            // stage the live instances' records
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
                const uint32_t t0 = (uint32_t)(tbase + (uint64_t)(R.y0 * TX + R.x0));
                const uint32_t w = (uint32_t)(R.x1 - R.x0), h = (uint32_t)(R.y1 - R.y0);
                s_a0[wave][e] = t0;
                s_a1[wave][e] = w;
                if (COUNT) A.comp[cbase + e] = make_uint4(t0, w | (h << 16), depth_bits, s_a5[wave][e]);
            }
            if (COUNT && lane == 0) A.comp_n[tile * kEmitWaves + wave] = n_live;
            __builtin_amdgcn_wave_barrier();
        }
        if (WIN) {
            // the views this block draws: from the first live entry of its
            // first non-empty wave to the last of its last (views increase
            // with the instance index)
            if (lane == 0) {
                const uint32_t T32 = (uint32_t)A.T;
                s_vmin[par][wave] = n_live ? (SCATTER ? s_a0[wave][0] / T32 : s_a4[wave][0]) : 0xFFFFFFFFu;
                s_vmax[par][wave] = n_live ? (SCATTER ? s_a0[wave][n_live - 1] / T32 : s_a4[wave][n_live - 1]) : 0u;
            }
            __syncthreads();  // also: every wave is done with the previous block's keys
            uint32_t vmin = 0xFFFFFFFFu, vmax = 0u;
            for (int k = 0; k < kEmitWaves; ++k) {
                vmin = min(vmin, s_vmin[par][k]);
                vmax = max(vmax, s_vmax[par][k]);
            }
            if (vmin != 0xFFFFFFFFu && (win_lo < 0 || (int64_t)vmax >= win_lo + A.win_views)) {
                // move the window to start at the block's first view (views
                // never go back): the views that leave are handed over, the
                // views that enter are set up, the ones in both keep their slots
                const int64_t old_hi = win_lo < 0 ? (int64_t)vmin : win_lo + A.win_views;
                const int64_t lo = vmin, hi = lo + A.win_views;
                if (MODE == kEmitCountWin && win_lo >= 0) window_views(win_lo, old_hi < lo ? old_hi : lo);
                if (MODE == kEmitScatterWin) window_views(old_hi > lo ? old_hi : lo, hi);
                win_lo = lo;
                win_base = (uint32_t)(lo * A.T);
                ring_off = (uint32_t)(lo % A.win_views) * (uint32_t)A.T;
                __syncthreads();
            }
        }
        // the wave's keys, 64 at a time: list starts increase strictly, so the
        // owner of key j is the last entry whose start is <= j.  The entries
        // that start inside a window [j0, j0 + 64) are the (at most 64) ones
        // after the owner of key j0 - 1; each marks its first key's lane, and
        // a lane's owner is that owner plus the marks at or below it.
        if (n_live) {
            const uint32_t lim = (int64_t)wave_total < room ? wave_total : (uint32_t)room;
            int32_t cur = -1;  // owner of key j0 - 1 (uniform)
            for (uint32_t j0 = 0; j0 < lim; j0 += 64) {
                ++tag;
                const uint32_t e = (uint32_t)(cur + 1) + (uint32_t)lane;
                if (e < n_live) {
                    const uint32_t st = s_a6[wave][e];
                    if (st < j0 + 64u) s_flag[wave][st - j0] = tag;
                }
                __builtin_amdgcn_wave_barrier();
                const uint64_t marks = __ballot(s_flag[wave][lane] == tag);
                const int lo = cur + (int)__popcll(marks & ((2ull << lane) - 1ull));
                cur += (int)__popcll(marks);
                const uint32_t j = j0 + (uint32_t)lane;
                if (j >= lim) continue;
                const uint32_t rel = j - s_a6[wave][lo], w = s_a1[wave][lo];
                const uint32_t tg = s_a0[wave][lo] + (rel / w) * (uint32_t)TX + rel % w;  // tile across all views
                if (MODE == kEmitSortKeys) {
                    const int64_t k = kw + (int64_t)j;
                    A.keys[k] = ((uint64_t)tg << 32) | (uint64_t)s_a2[wave][lo];
                    A.vals[k] = s_a5[wave][lo];
                } else if (MODE == kEmitCountTiles) {
                    atomicAdd(s_aux + tg, 1u);
                } else if (MODE == kEmitScatterTiles) {
                    const uint32_t slot = atomicAdd(s_aux + tg, 1u);
                    A.bucket[slot] = ((uint64_t)s_a2[wave][lo] << 32) | (uint64_t)s_a5[wave][lo];
                } else {
                    const uint32_t rel = tg - win_base;  // in the window when below win_tiles
                    uint32_t ring = rel + ring_off;
                    if (ring >= win_tiles) ring -= win_tiles;
                    if (MODE == kEmitCountWin) {
                        if (rel < win_tiles) atomicAdd(s_aux + ring, 1u);
                        else atomicAdd(A.tile_over + tg, 1u);
                    } else {
                        // keys outside the window take the tile's last slots,
                        // handed out counting the overflow back down to zero
                        const uint32_t slot = rel < win_tiles
                                                  ? atomicAdd(s_aux + ring, 1u)
                                                  : A.tile_start[tg] + A.tile_count[tg] + atomicSub(A.tile_over + tg, 1u) - 1u;
                        A.bucket[slot] = ((uint64_t)s_a2[wave][lo] << 32) | (uint64_t)s_a5[wave][lo];
                    }
                }
            }
        }
        // sort keys: s_wsum is reused by the next tile (the other modes keep
        // only per-wave state between tiles)
        if (MODE == kEmitSortKeys) __syncthreads();
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
    if (MODE == kEmitCountWin && win_lo >= 0) {
        __syncthreads();
        window_views(win_lo, win_lo + A.win_views);
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

// Tile sorts by bucket length (class: list part and kernel): up to
// kTinySortCap entries one wave (class 4, eight entries per thread), up to
// kSmallSortCap a 256-thread workgroup (class 3, eight each), up to
// kMidSortCap a 256-thread workgroup (class 2, sixteen each, four resident
// per CU), up to kLargeSortCap a 512-thread workgroup (class 1, sixteen
// each, two per CU), longer ones a 1024-thread workgroup (class 0, sixteen
// each: kTileSortCap in LDS, beyond that runs and merges).
constexpr int kTinySortCap = 512;
constexpr int kSmallSortBlock = 256, kSmallSortCap = 2048, kMidSortCap = 4096;
constexpr int kLargeSortBlock = 512, kLargeSortCap = 8192;
constexpr int kTileSortBlock = 1024, kTileSortCap = 16384;
constexpr int kSortClasses = 5;

// Exclusive scan of the tile totals (one workgroup): the key count and the
// overflow flag (count above the capacity), each tile's first key, the
// ranges ([first, end) for tiles with keys, [0, 0) otherwise, and all [0, 0)
// after an overflow), the compositing work order, and the lists the tile
// sorts take their tiles from: sort_list holds the tiles of more than
// kLargeSortCap keys by descending length (in bins of 1024 keys), then those
// of the four shorter classes, longest class first; sort_ctl holds the five
// counts, the number of tiles of more than kTileSortCap keys and of their runs
// of up to kTileSortCap keys, which run_list holds as {tile, run}.  Counts are read coalesced, a chunk of
// up to kScanChunk tiles at a time, into LDS.
constexpr int kScanChunk = 16384;
constexpr int kSortBins = 64;
constexpr int kHugeBins = kSortBins - kTileSortCap / 1024;  // the bins of the tiles longer than kTileSortCap
// sort_ctl: the five class counts, then the number of tiles longer than
// kTileSortCap (the first ones of the list) and of their runs
constexpr int kSortCtlWords = kSortClasses + 2;

// the list bin of a tile: 0 = longest .. kSortBins - 1, then kSortBins +
// 0 .. 3 for the four shorter classes
__device__ __forceinline__ uint32_t sort_bin(uint32_t len) {
    if (len <= (uint32_t)kTinySortCap) return kSortBins + 3;
    if (len <= (uint32_t)kSmallSortCap) return kSortBins + 2;
    if (len <= (uint32_t)kMidSortCap) return kSortBins + 1;
    if (len <= (uint32_t)kLargeSortCap) return kSortBins;
    const uint32_t k = (len - 1u) >> 10;  // a tile of more than kTileSortCap keys lands below kHugeBins
    return (uint32_t)(kSortBins - 1) - (k < (uint32_t)(kSortBins - 1) ? k : (uint32_t)(kSortBins - 1));
}

// One slot per active lane from *counter (lanes in order): one LDS atomic
// for the wave.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool active) {
    const int lane = threadIdx.x & 63;
    const uint64_t m = __ballot(active);
    if (!m) return 0u;  // uniform
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t b = 0u;
    if (lane == leader) b = atomicAdd(counter, (uint32_t)__popcll(m));
    b = __builtin_amdgcn_readlane(b, leader);
    return b + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

template <int PER>
__global__ void __launch_bounds__(1024) bucket_tilescan_kernel(const uint32_t *tile_count, const uint32_t *tile_over,
                                                               int64_t n_tiles, int64_t capacity, uint32_t *tile_start,
                                                               uint32_t *ranges, uint32_t *order, uint32_t *sort_list,
                                                               uint32_t *sort_ctl, uint2 *run_list, int64_t *d_num,
                                                               int32_t *d_overflow) {
    constexpr int CH = PER * 1024;  // tiles per chunk
    __shared__ uint32_t s_runs;
    __shared__ uint32_t s_c[CH];
    __shared__ uint32_t s_st[CH];  // first keys of the chunk's tiles
    __shared__ uint64_t s_w[16];
    __shared__ uint32_t s_cnt[kOrderQueues][kOrderBins];
    __shared__ uint32_t s_big[kSortBins + kSortClasses - 1];  // long tiles by bin, then the shorter classes
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n_chunks = (n_tiles + CH - 1) / CH;
    // keys per tile: the counted ones, plus those counted outside a window;
    // s_c[k] = count of tile cb + k (0 past the end), loads in flight together
    int64_t loaded = -1;
    auto load_chunk = [&](int64_t cb) {
        if (loaded == cb) return;  // uniform
        __syncthreads();
        // every load issued before any is used: addresses clamped in bounds,
        // counts past the end zeroed afterwards
        uint32_t c[PER], o[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t t = min(cb + k * 1024 + tid, n_tiles - 1);
            c[k] = tile_count[t];
            o[k] = tile_over ? tile_over[t] : 0u;
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) s_c[k * 1024 + tid] = cb + k * 1024 + tid < n_tiles ? c[k] + o[k] : 0u;
        loaded = cb;
        __syncthreads();
    };
    for (int i = tid; i < kOrderQueues * kOrderBins; i += 1024) (&s_cnt[0][0])[i] = 0u;
    if (tid < kSortBins + kSortClasses - 1) s_big[tid] = 0u;
    if (tid == 0) s_runs = 0u;
    // 1. the total, so that the overflow is known before anything is written
    // (one chunk: the scan below finds it before its first store)
    uint64_t total = 0u;
    for (int64_t ch = 0; n_chunks > 1 && ch < n_chunks; ++ch) {
        load_chunk(ch * CH);
        uint64_t sum = 0u;
#pragma unroll
        for (int k = 0; k < PER; ++k) sum += s_c[k * 1024 + tid];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) sum += __shfl_xor(sum, off, 64);
        __syncthreads();
        if (lane == 0) s_w[wave] = sum;
        __syncthreads();
        for (int k = 0; k < 16; ++k) total += s_w[k];
    }
    bool ovf = total > (uint64_t)capacity;  // then every range is [0, 0) and nothing is listed
    // 2. starts and ranges (each thread PER consecutive tiles), then the bin
    // counts (consecutive tiles on consecutive lanes: the order's queues and
    // bins spread over the lanes)
    uint64_t carry = 0u;
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
        const int64_t cb = ch * CH;
        load_chunk(cb);
        uint32_t c[PER];
        uint64_t sum = 0u;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            c[k] = s_c[tid * PER + k];
            sum += c[k];
        }
        uint64_t incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        __syncthreads();  // s_w of the previous chunk is read
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint64_t run = carry + incl - sum, chunk_total = 0u;
        for (int k = 0; k < 16; ++k) {
            if (k < wave) run += s_w[k];
            chunk_total += s_w[k];
        }
        carry += chunk_total;
        if (n_chunks == 1) ovf = carry > (uint64_t)capacity;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            s_st[tid * PER + k] = (uint32_t)run;
            run += c[k];
        }
        __syncthreads();
        // consecutive tiles on consecutive lanes: coalesced stores
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (cb + k * 1024 >= n_tiles) break;  // uniform: nothing left in the chunk
            const int64_t t = cb + k * 1024 + tid;
            if (t < n_tiles) {
                const uint32_t c1 = s_c[k * 1024 + tid], st = s_st[k * 1024 + tid];
                const bool has = c1 && !ovf;
                tile_start[t] = st;
                reinterpret_cast<uint2 *>(ranges)[t] = has ? make_uint2(st, st + c1) : make_uint2(0u, 0u);
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (cb + k * 1024 >= n_tiles) break;  // uniform
            const int64_t t = cb + k * 1024 + tid;
            const uint32_t c1 = ovf ? 0u : s_c[k * 1024 + tid];
            if (order && t < n_tiles) atomicAdd(&s_cnt[t % kOrderQueues][order_bin(c1)], 1u);
            const uint32_t bin = sort_bin(c1);
            if (c1 && bin < (uint32_t)kSortBins) atomicAdd(&s_big[bin], 1u);
#pragma unroll
            for (int cl = 0; cl < kSortClasses - 1; ++cl) {
                const uint64_t m = __ballot(c1 && bin == (uint32_t)(kSortBins + cl));
                if (lane == 0 && m) atomicAdd(&s_big[kSortBins + cl], (uint32_t)__popcll(m));
            }
        }
    }
    if (tid == 0) {
        *d_num = (int64_t)carry;
        *d_overflow = ovf ? 1 : 0;
    }
    // 3. bin starts, then the order and the sort lists
    if (order) order_bin_starts(s_cnt);
    __syncthreads();
    if (wave == 0) {
        const uint32_t b = s_big[lane];
        uint32_t incl = b;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        s_big[lane] = incl - b;
        const uint32_t n_huge = __shfl(incl - b, kHugeBins, 64);
        if (lane == 0) sort_ctl[kSortClasses] = n_huge;
        if (lane == 63) {
            // the shorter classes follow the long tiles, in order
            uint32_t at = incl;
            sort_ctl[0] = incl;
            for (int cl = 0; cl < kSortClasses - 1; ++cl) {
                const uint32_t cnt = s_big[kSortBins + cl];
                sort_ctl[1 + cl] = cnt;
                s_big[kSortBins + cl] = at;
                at += cnt;
            }
        }
    }
    __syncthreads();
    const int64_t qs = order_stride(n_tiles);
    for (int64_t ch = 0; ch < n_chunks; ++ch) {
        const int64_t cb = ch * CH;
        load_chunk(cb);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (cb + k * 1024 >= n_tiles) break;  // uniform
            const int64_t t = cb + k * 1024 + tid;
            const bool in = t < n_tiles;
            const uint32_t c = (ovf || !in) ? 0u : s_c[k * 1024 + tid];
            if (order && in) {
                const int q = (int)(t % kOrderQueues);
                order[q * qs + atomicAdd(&s_cnt[q][order_bin(c)], 1u)] = (uint32_t)t;
            }
            const uint32_t bin = sort_bin(c);
            uint32_t slot = 0u;
#pragma unroll
            for (int cl = 0; cl < kSortClasses - 1; ++cl) {
                const uint32_t y = wave_append(&s_big[kSortBins + cl], c && bin == (uint32_t)(kSortBins + cl));
                if (bin == (uint32_t)(kSortBins + cl)) slot = y;
            }
            if (c) sort_list[bin < (uint32_t)kSortBins ? atomicAdd(&s_big[bin], 1u) : slot] = (uint32_t)t;
            if (c > (uint32_t)kTileSortCap) {
                const uint32_t R = (c + kTileSortCap - 1) / kTileSortCap, r0 = atomicAdd(&s_runs, R);
                for (uint32_t r = 0; r < R; ++r) run_list[r0 + r] = make_uint2((uint32_t)t, r);
            }
        }
    }
    __syncthreads();
    if (tid == 0) sort_ctl[kSortClasses + 1] = s_runs;
}


// the tile scan with chunks of PER * 1024 tiles: the smallest that holds
// every tile, up to kScanChunk
static hipError_t launch_tilescan(const uint32_t *tile_count, const uint32_t *tile_over, int64_t n_tiles,
                                  int64_t capacity, uint32_t *tile_start, uint32_t *ranges, uint32_t *order,
                                  uint32_t *sort_list, uint32_t *sort_ctl, uint2 *run_list, int64_t *d_num,
                                  int32_t *d_overflow, hipStream_t s) {
#define GS_TILESCAN(P)                                                                                          \
    launch_kernel(bucket_tilescan_kernel<P>, dim3(1), dim3(1024), s, tile_count, tile_over, n_tiles, capacity, \
                  tile_start, ranges, order, sort_list, sort_ctl, run_list, d_num, d_overflow)
    if (n_tiles <= 1024) return GS_TILESCAN(1);
    if (n_tiles <= 2048) return GS_TILESCAN(2);
    if (n_tiles <= 4096) return GS_TILESCAN(4);
    return GS_TILESCAN(kScanChunk / 1024);
#undef GS_TILESCAN
}

__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ascending sorting network (bitonic) over N registers, all indices fixed at
// compile time.
template <int N>
__device__ __forceinline__ void sort_regs(uint64_t (&v)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t x = v[i], y = v[l];
                    const bool sw = ((i & k) == 0) ? (x > y) : (x < y);
                    v[i] = sw ? y : x;
                    v[l] = sw ? x : y;
                }
            }
}

// Block merge sort of the L entries at in[0, L) (L <= NT * ITEMS; entries
// distinct and below ~0, which pads) with NT threads (tid < NT; NT = 64 and
// ONE_WAVE for a wave on its own).  The smallest power-of-two number of
// threads that holds L takes ITEMS consecutive entries each and sorts them
// in registers; then sorted runs are merged pairwise, each thread finding
// where its ITEMS outputs start on the merge path of its pair by a binary
// search in LDS and merging them into registers, until one run is left.  s
// holds n + n / ITEMS entries (n = NT * ITEMS; slot i + i / ITEMS keeps the
// per-thread rows free of bank conflicts).  Writes key (thi | depth bits) and
// value (instance) of sorted entry p to keys[p], vals[p], or the entry itself
// to raw[p] when raw is non-NULL; reads and writes are coalesced through LDS.
template <int NT, int ITEMS, bool ONE_WAVE>
__device__ __forceinline__ void merge_sort_lds(uint64_t *s, const uint64_t *in, uint32_t L, uint64_t thi,
                                               uint64_t *keys, uint32_t *vals, uint64_t *raw, uint32_t tid) {
    auto slot = [](uint32_t i) { return i + i / ITEMS; };
    auto sync = [] {
        if (ONE_WAVE) lds_wave_sync();
        else __syncthreads();
    };
    uint32_t nt = 1;
    while (nt * ITEMS < L) nt <<= 1;
    const uint32_t n = nt * ITEMS;
    const bool act = tid < nt;
    {
        // every load issued before any is used (clamped in bounds: L >= 1)
        uint64_t x[ITEMS];
#pragma unroll
        for (int m = 0; m < ITEMS; ++m) x[m] = in[min((uint32_t)m * NT + tid, L - 1u)];
#pragma unroll
        for (int m = 0; m < ITEMS; ++m) {
            const uint32_t i = (uint32_t)m * NT + tid;
            if (i < n) s[slot(i)] = i < L ? x[m] : ~0ull;
        }
    }
    sync();
    uint64_t v[ITEMS];
    if (act) {
#pragma unroll
        for (int m = 0; m < ITEMS; ++m) v[m] = s[slot(tid * ITEMS + m)];
        sort_regs<ITEMS>(v);
    }
    for (uint32_t R = ITEMS; R < n; R <<= 1) {  // uniform
        sync();  // the previous level's reads are done
        if (act) {
#pragma unroll
            for (int m = 0; m < ITEMS; ++m) s[slot(tid * ITEMS + m)] = v[m];
        }
        sync();
        if (act) {
            // runs A = [a0, a0 + R) and B = [a0 + R, a0 + 2R); this thread
            // writes outputs d .. d + ITEMS - 1 of their merge (ties: A first)
            const uint32_t p0 = tid * ITEMS, a0 = p0 & ~(2 * R - 1), b0 = a0 + R, d = p0 - a0;
            uint32_t lo = d > R ? d - R : 0u, hi = d < R ? d : R;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s[slot(a0 + mid)] <= s[slot(b0 + d - 1 - mid)]) lo = mid + 1;
                else hi = mid;
            }
            uint32_t i = lo, j = d - lo;
            uint64_t a = s[slot(a0 + min(i, R - 1))], b = s[slot(b0 + min(j, R - 1))];
#pragma unroll
            for (int m = 0; m < ITEMS; ++m) {
                const bool ta = j >= R || (i < R && a <= b);
                v[m] = ta ? a : b;
                i += ta ? 1u : 0u;
                j += ta ? 0u : 1u;
                if (m + 1 < ITEMS) {
                    const uint64_t x = s[slot(ta ? a0 + min(i, R - 1) : b0 + min(j, R - 1))];
                    a = ta ? x : a;
                    b = ta ? b : x;
                }
            }
        }
    }
    sync();
    if (act) {
#pragma unroll
        for (int m = 0; m < ITEMS; ++m) s[slot(tid * ITEMS + m)] = v[m];
    }
    sync();
    uint64_t x[ITEMS];
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) x[m] = s[slot(min((uint32_t)m * NT + tid, n - 1u))];
#pragma unroll
    for (int m = 0; m < ITEMS; ++m) {
        const uint32_t i = (uint32_t)m * NT + tid;
        if (i < L) {
            if (raw) {
                raw[i] = x[m];
            } else {
                keys[i] = thi | (x[m] >> 32);
                vals[i] = (uint32_t)x[m];
            }
        }
    }
}

// dst[i] = f(src[i]) for i < cnt by NT threads, eight loads in flight per
// thread (clamped in bounds) before their stores
template <int NT, typename F>
__device__ __forceinline__ void copy_block(const uint64_t *src, uint32_t cnt, uint32_t tid, F &&store) {
    for (uint32_t b0 = 0; b0 < cnt; b0 += 8u * NT) {
        uint64_t x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = src[min(b0 + (uint32_t)u * NT + tid, cnt - 1u)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = b0 + (uint32_t)u * NT + tid;
            if (i < cnt) store(i, x[u]);
        }
    }
}

// Merges the ascending runs A[0, la) and B[0, lb) (no two entries equal)
// into dst[0, la + lb) with NT threads, CHUNK outputs at a time: the next
// CHUNK entries of each run are staged in LDS (s holds 2 CHUNK), every
// thread finds where its stretch of the chunk starts on the merge path by a
// binary search in LDS and merges it (store(k, entry) for output k), and the
// thread whose stretch ends the chunk tells how far the chunk got into A.
template <int NT, int CHUNK, typename Store>
__device__ __forceinline__ void merge_runs(const uint64_t *A, uint32_t la, const uint64_t *Bv, uint32_t lb,
                                           Store &&store, uint64_t *s, uint32_t *s_take, uint32_t tid) {
    constexpr uint32_t PER = CHUNK / NT;
    uint64_t *sA = s, *sB = s + CHUNK;
    // i = how many of the first d merged entries come from sA[0, na): the
    // least i with sA[i] > sB[d - 1 - i], else min(d, na)
    auto split = [&](uint32_t d, uint32_t na, uint32_t nb) {
        uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
        while (lo < hi) {
            const uint32_t i = (lo + hi) >> 1;
            if (sA[i] < sB[d - 1 - i]) lo = i + 1;
            else hi = i;
        }
        return lo;
    };
    uint32_t i0 = 0, j0 = 0;
    while (i0 + j0 < la + lb) {  // uniform
        const uint32_t na = min((uint32_t)CHUNK, la - i0), nb = min((uint32_t)CHUNK, lb - j0);
        const uint32_t m = min((uint32_t)CHUNK, na + nb);
        if (na) copy_block<NT>(A + i0, na, tid, [&](uint32_t k, uint64_t x) { sA[k] = x; });
        if (nb) copy_block<NT>(Bv + j0, nb, tid, [&](uint32_t k, uint64_t x) { sB[k] = x; });
        __syncthreads();
        const uint32_t d0 = min(m, tid * PER), d1 = min(m, d0 + PER);
        if (d0 < d1) {
            uint32_t i = split(d0, na, nb), j = d0 - i;
            for (uint32_t d = d0; d < d1; ++d) {
                const bool take_a = j >= nb || (i < na && sA[i] < sB[j]);
                store(i0 + j0 + d, take_a ? sA[i++] : sB[j++]);
            }
            if (d1 == m) *s_take = i;  // the thread that ends the chunk knows how far it got into A
        }
        __syncthreads();
        const uint32_t ta = *s_take;
        i0 += ta;
        j0 += m - ta;
        __syncthreads();  // sA, sB and s_take are reused by the next chunk
    }
}

// Levels of pairwise merging a tile of L > CAP entries takes (runs of CAP
// entries); with an odd count the runs are sorted into the bucket, else into
// the key array, so that the last level reads the bucket and writes the keys.
template <int CAP>
__device__ __forceinline__ bool runs_in_bucket(uint32_t L) {
    int levels = 0;
    for (uint32_t w = (uint32_t)CAP; w < L; w <<= 1) ++levels;
    return levels & 1;
}

// A tile of L > CAP entries whose runs of CAP entries are sorted, raw, at
// bucket[b ..] or keys[b ..] (runs_in_bucket): runs merged pairwise by the
// workgroup, ping-ponging between the two, the last level writing keys
// (tile << 32 | depth bits) and values (s: CAP entries of LDS).
template <int THREADS, int CAP>
__device__ __forceinline__ void merge_tile_runs(uint64_t *bucket, uint64_t *keys, uint32_t *vals, uint32_t tile,
                                                uint32_t b, uint32_t L, uint64_t *s, uint32_t *s_take) {
    const uint64_t thi = (uint64_t)tile << 32;
    const bool in_bucket = runs_in_bucket<CAP>(L);
    uint64_t *src = in_bucket ? bucket + b : keys + b, *dst = in_bucket ? keys + b : bucket + b;
    uint64_t *kk = keys + b;
    uint32_t *vv = vals + b;
    for (uint32_t w = (uint32_t)CAP; w < L; w <<= 1) {
        const bool last = 2u * w >= L;  // one pair left: its merge writes the keys
        for (uint32_t a0 = 0; a0 < L; a0 += 2 * w) {
            const uint32_t la = min(w, L - a0), lb = min(w, L - a0 - la);
            if (lb == 0u) {  // never on the last level
                uint64_t *d = dst + a0;
                copy_block<THREADS>(src + a0, la, threadIdx.x, [&](uint32_t i, uint64_t x) { d[i] = x; });
            } else if (last) {
                merge_runs<THREADS, CAP / 2>(src + a0, la, src + a0 + la, lb,
                                             [&](uint32_t k, uint64_t c) {
                                                 kk[a0 + k] = thi | (c >> 32);
                                                 vv[a0 + k] = (uint32_t)c;
                                             },
                                             s, s_take, threadIdx.x);
            } else {
                uint64_t *d = dst + a0;
                merge_runs<THREADS, CAP / 2>(src + a0, la, src + a0 + la, lb,
                                             [&](uint32_t k, uint64_t x) { d[k] = x; }, s, s_take, threadIdx.x);
            }
        }
        __syncthreads();
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
}

// One workgroup per item, items taken in rounds from the part of the list
// the tile scan made for CLASS (class 0 longest first): a bucket of up to CAP
// entries sorted in LDS, its keys (tile << 32 | depth bits) and values
// (instance) written to the tile's range.  Besides the five classes, two
// groupings for launches of few tiles, where one launch for several classes
// keeps every tile in flight at once: kSortShort (classes 3 and 4, up to 2048
// entries, 256 threads: their 18 KB of LDS let eight workgroups share a CU,
// so 2048 tiles sort in one round) and kSortLong (classes 0..2, 1024 threads,
// a tile longer than CAP sorted as runs and merged by its own workgroup).  With sixteen
// entries per thread, a bucket that fits eight per thread takes eight (more
// threads at work).
constexpr int kSortShort = 5, kSortLong = 6;

template <int THREADS, int CAP, int CLASS>
__global__ void __launch_bounds__(THREADS) tile_sort_kernel(uint64_t *bucket, const uint32_t *ranges,
                                                            const uint32_t *sort_list, const uint32_t *sort_ctl,
                                                            const uint2 *run_list, uint64_t *keys, uint32_t *vals,
                                                            const int32_t *d_overflow) {
    __shared__ uint64_t s[CAP + CAP / 8];
    __shared__ uint32_t s_take;
    if (*d_overflow) return;
    // class 0: first the runs of the tiles longer than CAP (sorted here, raw,
    // into the key array; the merge kernel finishes those tiles), then the
    // other tiles
    constexpr bool SMALL = CLASS != 0;
    constexpr int C0 = CLASS == kSortShort ? 3 : CLASS == kSortLong ? 0 : CLASS;
    constexpr int C1 = CLASS == kSortShort ? 4 : CLASS == kSortLong ? 2 : CLASS;
    uint32_t first = 0u, n_tiles = 0u;
    for (int c = 0; c < C0; ++c) first += sort_ctl[c];
    for (int c = C0; c <= C1; ++c) n_tiles += sort_ctl[c];
    const uint32_t n_huge = SMALL ? 0u : sort_ctl[kSortClasses], n_runs = SMALL ? 0u : sort_ctl[kSortClasses + 1];
    const uint32_t n_items = n_runs + n_tiles - n_huge;
    const uint32_t G = gridDim.x;
    for (uint32_t r0 = 0; r0 < n_items; r0 += G) {  // uniform
        // rounds of G items; class 0 comes longest first, so its rounds
        // alternate direction to even out the workgroups' totals
        const uint32_t idx = r0 + (SMALL || ((r0 / G) & 1u) == 0u ? blockIdx.x : G - 1u - blockIdx.x);
        if (idx >= n_items) continue;
        if (!SMALL && idx < n_runs) {
            const uint2 tr = run_list[idx];
            const uint32_t b = ranges[2 * tr.x], L = ranges[2 * tr.x + 1] - b, off = tr.y * (uint32_t)CAP;
            merge_sort_lds<THREADS, CAP / THREADS, false>(s, bucket + b + off, min((uint32_t)CAP, L - off), 0ull,
                                                          nullptr, nullptr,
                                                          (runs_in_bucket<CAP>(L) ? bucket : keys) + b + off,
                                                          threadIdx.x);
        } else {
            const uint32_t tile = sort_list[first + n_huge + (idx - n_runs)];
            const uint32_t b = ranges[2 * tile], L = ranges[2 * tile + 1] - b;
            constexpr int IT = CAP / THREADS;
            if (CLASS == kSortLong && L > (uint32_t)CAP) {
                for (uint32_t off = 0; off < L; off += (uint32_t)CAP) {
                    merge_sort_lds<THREADS, IT, false>(s, bucket + b + off, min((uint32_t)CAP, L - off), 0ull, nullptr,
                                                       nullptr, (runs_in_bucket<CAP>(L) ? bucket : keys) + b + off,
                                                       threadIdx.x);
                    __syncthreads();  // s is reused by the next run
                }
                merge_tile_runs<THREADS, CAP>(bucket, keys, vals, tile, b, L, s, &s_take);
            } else if (IT == 16 && L <= (uint32_t)(THREADS * 8))
                merge_sort_lds<THREADS, (IT == 16 ? 8 : IT), false>(s, bucket + b, L, (uint64_t)tile << 32, keys + b,
                                                                    vals + b, nullptr, threadIdx.x);
            else
                merge_sort_lds<THREADS, IT, false>(s, bucket + b, L, (uint64_t)tile << 32, keys + b, vals + b, nullptr,
                                                   threadIdx.x);
        }
        __syncthreads();  // s is reused by the next item
    }
}

// The tiles longer than CAP, one workgroup each: their sorted runs (raw in
// the key array) merged pairwise, ping-ponging between the key array and the
// bucket, then written as keys (tile << 32 | depth bits) and values.
template <int THREADS, int CAP>
__global__ void __launch_bounds__(THREADS) tile_merge_kernel(uint64_t *bucket, const uint32_t *ranges,
                                                             const uint32_t *sort_list, const uint32_t *sort_ctl,
                                                             uint64_t *keys, uint32_t *vals,
                                                             const int32_t *d_overflow) {
    __shared__ uint64_t s[CAP];
    __shared__ uint32_t s_take;
    if (*d_overflow) return;
    const uint32_t n_huge = sort_ctl[kSortClasses];
    for (uint32_t h = blockIdx.x; h < n_huge; h += gridDim.x) {  // uniform
        const uint32_t tile = sort_list[h];
        const uint32_t b = ranges[2 * tile], L = ranges[2 * tile + 1] - b;
        merge_tile_runs<THREADS, CAP>(bucket, keys, vals, tile, b, L, s, &s_take);
        __syncthreads();  // s is reused by the next tile
    }
}

// The tiles of 1..kTinySortCap keys: one wave each, four waves per
// workgroup, waves striding over the list (no workgroup barriers).
__global__ void __launch_bounds__(256) tile_sort_wave_kernel(uint64_t *bucket, const uint32_t *ranges,
                                                             const uint32_t *sort_list, const uint32_t *sort_ctl,
                                                             uint64_t *keys, uint32_t *vals,
                                                             const int32_t *d_overflow) {
    constexpr int SLOTS = kTinySortCap + kTinySortCap / 8;
    __shared__ uint64_t s[4][SLOTS];
    if (*d_overflow) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t first = 0u;
    for (int c = 0; c < kSortClasses - 1; ++c) first += sort_ctl[c];
    const uint32_t n_mine = sort_ctl[kSortClasses - 1];
    for (uint32_t idx = blockIdx.x * 4u + (uint32_t)wave; idx < n_mine; idx += gridDim.x * 4u) {  // uniform per wave
        const uint32_t tile = sort_list[first + idx];
        const uint32_t b = ranges[2 * tile], L = ranges[2 * tile + 1] - b;
        merge_sort_lds<64, kTinySortCap / 64, true>(s[wave], bucket + b, L, (uint64_t)tile << 32, keys + b, vals + b,
                                                    nullptr, (uint32_t)lane);
        lds_wave_sync();  // s is reused by the next tile
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

SortPlan make_sort_plan(int64_t n, int64_t capacity, int64_t tiles_per_view, int64_t n_views) {
    SortPlan p;
    const int64_t n_tiles_total = tiles_per_view * n_views;
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
    // bucket path: per-workgroup tile counters, tile totals (and, windowed,
    // the keys counted outside a window right after them) and starts; the
    // counters of up to kBucketMaxTiles tiles fit in LDS, beyond that a
    // window of whole views does when a view has at most kLdsTiles tiles
    p.T = tiles_per_view;
    p.windowed = n_tiles_total > kBucketMaxTiles;
    p.win_views = (int)(kLdsTiles / (tiles_per_view > 0 ? tiles_per_view : 1));
    p.bucket_ok = !p.windowed || (tiles_per_view <= kLdsTiles && tiles_per_view > 0 && n_tiles_total <= kWindowMaxTiles);
    const int64_t grid = p.windowed ? kWinGrid : kBucketGrid;
    p.bucket_blocks = p.scan_blocks < grid ? p.scan_blocks : grid;
    p.off_tcnt = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)p.bucket_blocks * (size_t)n_tiles_total);
    p.off_tcount = o;
    p.off_tover = o + sizeof(uint32_t) * (size_t)n_tiles_total;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)n_tiles_total * (p.windowed ? 2 : 1));
    p.off_tstart = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)n_tiles_total);
    // the count pass's compact records of the live instances
    p.off_comp = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * 4 * (size_t)kScanTile * (size_t)p.scan_blocks);
    p.off_compn = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)kEmitWaves * (size_t)p.scan_blocks);
    // the tile sorts' list of tiles and their counters
    p.off_slist = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * (size_t)n_tiles_total);
    p.off_sctl = o;
    if (p.bucket_ok) o = align256(o + sizeof(uint32_t) * kSortCtlWords);
    // the runs of the tiles longer than kTileSortCap (at most one per tile and one per kTileSortCap keys)
    p.off_rlist = o;
    if (p.bucket_ok)
        o = align256(o + sizeof(uint2) * (size_t)(n_tiles_total + (capacity > 0 ? capacity : 1) / kTileSortCap + 1));
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
    A.comp = reinterpret_cast<uint4 *>(ws + P.off_comp);
    A.comp_n = reinterpret_cast<uint32_t *>(ws + P.off_compn);
    uint32_t *tcount = reinterpret_cast<uint32_t *>(ws + P.off_tcount);
    uint32_t *tstart = reinterpret_cast<uint32_t *>(ws + P.off_tstart);
    uint32_t *slist = reinterpret_cast<uint32_t *>(ws + P.off_slist);
    uint32_t *sctl = reinterpret_cast<uint32_t *>(ws + P.off_sctl);
    uint2 *rlist = reinterpret_cast<uint2 *>(ws + P.off_rlist);
    if (P.windowed) {
        // window totals and the keys outside windows start at zero (one fill:
        // the two arrays are adjacent); the counters hold offsets after the count
        A.tile_count = tcount;
        A.tile_over = reinterpret_cast<uint32_t *>(ws + P.off_tover);
        A.T = P.T;
        A.win_views = P.win_views;
        if ((e = launch_fill_u32(tcount, 0u, 2 * P.n_tiles_total, s)) != hipSuccess) return e;
        if ((e = launch_kernel(emit_kernel<kEmitCountWin>, dim3((unsigned)P.bucket_blocks), dim3(kEmitBlock), s,
                               A)) != hipSuccess)
            return e;
        if ((e = launch_tilescan(tcount, A.tile_over, P.n_tiles_total, P.capacity, tstart, ranges, order, slist,
                                 sctl, rlist, d_num, d_overflow, s)) != hipSuccess)
            return e;
        if ((e = launch_kernel(emit_kernel<kEmitScatterWin>, dim3((unsigned)P.bucket_blocks), dim3(kEmitBlock), s,
                               A)) != hipSuccess)
            return e;
    } else {
        if ((e = launch_kernel(emit_kernel<kEmitCountTiles>, dim3((unsigned)P.bucket_blocks), dim3(kEmitBlock), s,
                               A)) != hipSuccess)
            return e;
        if ((e = launch_kernel(bucket_colscan_kernel, dim3((unsigned)((P.n_tiles_total + 3) / 4)), dim3(256), s,
                               A.tile_cnt, (int)P.bucket_blocks, P.n_tiles_total, tcount)) != hipSuccess)
            return e;
        if ((e = launch_tilescan(tcount, nullptr, P.n_tiles_total, P.capacity, tstart, ranges, order, slist, sctl,
                                 rlist, d_num, d_overflow, s)) != hipSuccess)
            return e;
        if ((e = launch_kernel(emit_kernel<kEmitScatterTiles>, dim3((unsigned)P.bucket_blocks), dim3(kEmitBlock), s,
                               A)) != hipSuccess)
            return e;
    }
    // the tile sorts take their tiles from the list in rounds of one per
    // workgroup (wave); few tiles: two launches cover every class, so all
    // tiles sort at once; many: one launch per class, each sized to fill the
    // chip with its own workgroups
    const uint32_t *cl = slist, *cc = sctl;
    const uint2 *rl = rlist;
    const int32_t *ov = d_overflow;
    const uint32_t *rg = ranges;
    auto grid = [&](int64_t per_cu, int64_t cap) {
        int64_t g = per_cu * (int64_t)n_cu;
        return (unsigned)(g < cap ? g : (cap > 0 ? cap : 1));
    };
    const int64_t nt = P.n_tiles_total;
    if (!P.windowed) {
        if ((e = launch_kernel(tile_sort_kernel<kSmallSortBlock, kSmallSortCap, kSortShort>, dim3(grid(8, nt)),
                               dim3(kSmallSortBlock), s, A.bucket, rg, cl, cc, rl, keys, vals, ov)) != hipSuccess)
            return e;
        return launch_kernel(tile_sort_kernel<kTileSortBlock, kTileSortCap, kSortLong>, dim3(grid(1, nt)),
                             dim3(kTileSortBlock), s, A.bucket, rg, cl, cc, rl, keys, vals, ov);
    }
    {
        if ((e = launch_kernel(tile_sort_wave_kernel, dim3(grid(8, (nt + 3) / 4)), dim3(256), s, A.bucket, rg, cl, cc,
                               keys, vals, ov)) != hipSuccess)
            return e;
        if ((e = launch_kernel(tile_sort_kernel<kSmallSortBlock, kSmallSortCap, 3>, dim3(grid(8, nt)),
                               dim3(kSmallSortBlock), s, A.bucket, rg, cl, cc, rl, keys, vals, ov)) != hipSuccess)
            return e;
        if ((e = launch_kernel(tile_sort_kernel<kSmallSortBlock, kMidSortCap, 2>, dim3(grid(4, nt)),
                               dim3(kSmallSortBlock), s, A.bucket, rg, cl, cc, rl, keys, vals, ov)) != hipSuccess)
            return e;
        if ((e = launch_kernel(tile_sort_kernel<kLargeSortBlock, kLargeSortCap, 1>, dim3(grid(2, nt)),
                               dim3(kLargeSortBlock), s, A.bucket, rg, cl, cc, rl, keys, vals, ov)) != hipSuccess)
            return e;
        if ((e = launch_kernel(tile_sort_kernel<kTileSortBlock, kTileSortCap, 0>, dim3(grid(1, 1ll << 40)),
                               dim3(kTileSortBlock), s, A.bucket, rg, cl, cc, rl, keys, vals, ov)) != hipSuccess)
            return e;
    }
    return launch_kernel(tile_merge_kernel<kTileSortBlock, kTileSortCap>, dim3(grid(1, 1ll << 40)),
                         dim3(kTileSortBlock), s, A.bucket, rg, cl, cc, keys, vals, ov);
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
