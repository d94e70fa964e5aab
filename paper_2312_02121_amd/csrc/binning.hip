// gs_bin_and_sort: tile binning and per-tile depth order (Sec. 2.2).
//
// The result is the list of (tile, depth, splat) entries sorted by the 64-bit key
// (global tile << 32) | float32 depth bits, equal keys in splat order -- the order a single
// stable LSD radix sort of those 64-bit keys produces. It is computed as two stable
// LDS-histogram radix sorts whose traffic does not grow with the 32 depth bits per entry:
//
//   1. depth sort of the P splats: 32-bit keys (float bits of t_z, culled splats last),
//      values = splat slot; four 8-bit passes over P keys. Ties keep slot order.
//   2. exclusive scan of tiles_touched in depth-rank order -> per-splat emit offsets and
//      K = total intersections (an overflow flag is raised when K exceeds the capacity).
//   3. emit in depth-rank order: each splat writes (global tile id, slot) for every tile of
//      its box, row-major. A lane emits its own splat when the box is small; splats with
//      large boxes (near the camera they can cover the whole image) are written by the
//      whole wave together, so one splat never serialises a thread over thousands of tiles.
//   4. stable sort of the K entries by tile id alone: ceil(log2(n_tiles) / 8) 8-bit passes
//      (two for 1920x1080 or 1280x720). Being stable, it keeps the depth-rank order inside
//      every tile. The last pass writes the splat slots to bins->ids and the 64-bit keys
//      (tile << 32 | depth bits of the slot) to bins->keys.
//   5. ranges: [start, end) of each tile's run; then the rasterizer's work list.
//
// Per entry this moves ~40 bytes where six 8-bit passes over 64-bit keys move ~190; for
// views with near-plane splats (hundreds of millions of entries) the sort is HBM-bound and
// the difference is the whole cost.
//
// Each pass is a per-block digit histogram, a scan of the digit-major histogram table and
// a stable scatter. Block ranking uses wave ballots to group equal digits and LDS counters
// per (wave, digit), so no LDS atomics contend on popular digits. Every kernel is sized
// from host-known capacities and reads its element count from device memory, so the whole
// sequence replays unchanged inside a captured HIP graph.
#include "common.h"

namespace gsx {

// ------------------------------------------------------------------------------ scan

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanBlock * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the exclusive prefix and the
// block total through *total.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *total)
{
    __shared__ T wave_tot[kScanBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    T incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T u = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += u;
    }
    if (lane == kWave - 1) wave_tot[wave] = incl;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / kWave; ++w) {
        const T x = wave_tot[w];
        if (w < wave) before += x;
        all += x;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// The scans read their input through a loader: load(i) returns element i (i < n).
template <typename T>
struct ArrayLoad {
    const T *p;
    __device__ T operator()(int64_t i) const { return p[i]; }
};

// tiles_touched of the splat at depth rank i
struct RankTiles {
    const int32_t *tiles;
    const int32_t *rank_ids;
    __device__ int64_t operator()(int64_t i) const { return tiles[rank_ids[i]]; }
};

template <typename Load, typename TAcc>
__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(Load in, int64_t n, TAcc *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    TAcc acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) acc += (TAcc)in(base + k);
    TAcc tot;
    block_exclusive_scan<TAcc>(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of sums[0..nb) in place; the grand total goes to *total
// (if not null) and, when cap >= 0, an overflow flag to *flag = (total > cap).
template <typename TAcc>
__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(TAcc *__restrict__ sums, int64_t nb,
                                                               int64_t *__restrict__ total,
                                                               int64_t *__restrict__ flag, int64_t cap)
{
    TAcc carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        const int64_t idx = base + threadIdx.x;
        const TAcc v = idx < nb ? sums[idx] : (TAcc)0;
        TAcc tot;
        const TAcc ex = block_exclusive_scan<TAcc>(v, &tot);
        if (idx < nb) sums[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (total) *total = (int64_t)carry;
        if (flag) *flag = (cap >= 0 && (int64_t)carry > cap) ? 1 : 0;
    }
}

template <typename Load, typename TAcc, typename TOut>
__global__ __launch_bounds__(kScanBlock) void scan_down_kernel(Load in, int64_t n, const TAcc *__restrict__ sums,
                                                               TOut *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    TAcc vals[kScanItems];
    TAcc acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = base + k < n ? (TAcc)in(base + k) : (TAcc)0;
        acc += vals[k];
    }
    TAcc tot;
    TAcc run = block_exclusive_scan<TAcc>(acc, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = (TOut)run;
        run += vals[k];
    }
}

static int64_t scan_blocks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

// Exclusive scan of n loaded values into out; sums needs scan_blocks(n) entries.
template <typename TAcc, typename TOut, typename Load>
static int scan_exclusive(Load in, int64_t n, TOut *out, TAcc *sums, int64_t *total, int64_t *flag, int64_t cap,
                          hipStream_t st)
{
    const int64_t nb = scan_blocks(n);
    if (nb == 0) return GS_OK;
    hipLaunchKernelGGL((scan_reduce_kernel<Load, TAcc>), dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, sums);
    hipLaunchKernelGGL((scan_sums_kernel<TAcc>), dim3(1), dim3(kScanBlock), 0, st, sums, nb, total, flag, cap);
    hipLaunchKernelGGL((scan_down_kernel<Load, TAcc, TOut>), dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n,
                       sums, out);
    return check_launch("scan");
}

// ------------------------------------------------------------------------ radix sort

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kSortItems = 16;                       // keys per lane
constexpr int kSortChunk = kSortBlock * kSortItems;  // keys per block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

__device__ inline int64_t sort_count(const int64_t *counter, int64_t cap)
{
    const int64_t k = *counter;
    return k < cap ? k : cap;
}

// Lanes of the wave whose `digit` equals this lane's, among lanes in `valid`.
__device__ inline uint64_t match_digit(unsigned digit, uint64_t valid)
{
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint64_t bal = __ballot((digit >> b) & 1u);
        peers &= ((digit >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

// Counts digits of this block's chunk. Wave w owns keys [w*M, (w+1)*M) of the chunk
// (M = kSortChunk / kSortWaves), walked in order so that ranks are stable.
__device__ inline void count_digits(const uint32_t (&key)[kSortItems], int64_t chunk_base, int64_t kvalid, int shift,
                                    unsigned (*cnt)[kRadix])
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = chunk_base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        const bool ok = idx < kvalid;
        const uint64_t valid = __ballot(ok);
        if (valid == 0) break;
        const unsigned d = (key[r] >> shift) & (kRadix - 1);
        const uint64_t peers = match_digit(d, valid);
        if (ok && (peers & lanemask_lt()) == 0) cnt[wave][d] += (unsigned)__popcll(peers);
    }
}

__global__ __launch_bounds__(kSortBlock) void radix_hist_kernel(const uint32_t *__restrict__ keys,
                                                                const int64_t *__restrict__ count, int64_t cap,
                                                                int shift, int nblocks, unsigned *__restrict__ hist)
{
    __shared__ unsigned cnt[kSortWaves][kRadix];
    for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortBlock) (&cnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t kvalid = sort_count(count, cap);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base < kvalid) {
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        uint32_t key[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
            key[r] = idx < kvalid ? keys[idx] : 0u;
        }
        count_digits(key, base, kvalid, shift, cnt);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kSortBlock) {
        unsigned s = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) s += cnt[w][d];
        hist[(int64_t)d * nblocks + blockIdx.x] = s;
    }
}

// hist_scan holds, digit-major, the exclusive prefix of the histogram table: the output
// position of the first key with digit d in block b. When keys64_out is set (the last tile
// pass), the scatter writes the 64-bit output key (tile << 32 | depth bits of the value)
// there instead of the 32-bit key.
__global__ __launch_bounds__(kSortBlock) void radix_scatter_kernel(const uint32_t *__restrict__ keys_in,
                                                                   const int32_t *__restrict__ vals_in,
                                                                   const int64_t *__restrict__ count, int64_t cap,
                                                                   int shift, int nblocks,
                                                                   const unsigned *__restrict__ hist_scan,
                                                                   uint32_t *__restrict__ keys_out,
                                                                   int32_t *__restrict__ vals_out,
                                                                   uint64_t *__restrict__ keys64_out,
                                                                   const float *__restrict__ depth)
{
    __shared__ unsigned cnt[kSortWaves][kRadix];
    const int64_t kvalid = sort_count(count, cap);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base >= kvalid) return;   // uniform over the block
    for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortBlock) (&cnt[0][0])[d] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t key[kSortItems];
    int32_t val[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        const bool ok = idx < kvalid;
        key[r] = ok ? keys_in[idx] : 0u;
        val[r] = ok ? vals_in[idx] : 0;
    }
    count_digits(key, base, kvalid, shift, cnt);
    __syncthreads();
    // turn counts into this block's per-(wave, digit) output cursors
    for (int d = threadIdx.x; d < kRadix; d += kSortBlock) {
        unsigned run = hist_scan[(int64_t)d * nblocks + blockIdx.x];
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const unsigned c = cnt[w][d];
            cnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        const bool ok = idx < kvalid;
        const uint64_t valid = __ballot(ok);
        if (valid == 0) break;
        const unsigned d = (key[r] >> shift) & (kRadix - 1);
        const uint64_t peers = match_digit(d, valid);
        const unsigned pos = cnt[wave][d] + (unsigned)__popcll(peers & lanemask_lt());
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & lanemask_lt()) == 0) cnt[wave][d] += (unsigned)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (ok) {
            vals_out[pos] = val[r];
            if (keys64_out)
                keys64_out[pos] = ((uint64_t)key[r] << 32) | (uint64_t)__float_as_uint(depth[val[r]]);
            else
                keys_out[pos] = key[r];
        }
    }
}

// ------------------------------------------------------------------- depth order, emit

// Depth keys of every splat: float bits of t_z (positive, so bit order is value order);
// culled splats get 0xffffffff and sort last. Thread 0 also stores the key count.
__global__ __launch_bounds__(256) void depth_keys_kernel(const int32_t *__restrict__ tiles,
                                                         const float *__restrict__ depth, int64_t n,
                                                         uint32_t *__restrict__ dkey, int32_t *__restrict__ dval,
                                                         int64_t *__restrict__ count)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *count = n;
    if (p >= n) return;
    dkey[p] = tiles[p] > 0 ? __float_as_uint(depth[p]) : 0xffffffffu;
    dval[p] = (int32_t)p;
}

// Splats whose box has at most this many tiles are emitted by their own lane.
constexpr int kEmitLaneMax = 16;

__device__ inline void emit_tiles(int64_t k0, int count_begin, int count_step, int n_tiles_box, const int4 &b,
                                  int toff, int tx_n, int32_t slot, int64_t cap, uint32_t *__restrict__ tkey,
                                  int32_t *__restrict__ tval)
{
    const int w = b.z - b.x + 1;
    for (int j = count_begin; j < n_tiles_box; j += count_step) {
        const int64_t k = k0 + j;
        if (k >= cap) break;
        const int ty = b.y + j / w, tx = b.x + j % w;
        tkey[k] = (uint32_t)(toff + ty * tx_n + tx);
        tval[k] = slot;
    }
}

// One thread per depth rank. Entries are written at the rank's scan offset, row-major over
// the box; entries beyond the capacity are dropped (the overflow flag is already set).
__global__ __launch_bounds__(256) void emit_kernel(const int32_t *__restrict__ rank_ids,
                                                   const int64_t *__restrict__ offsets,
                                                   const int32_t *__restrict__ tiles, const int4 *__restrict__ rect,
                                                   const gs_camera *__restrict__ cams, int n_cams, int64_t n_splats,
                                                   int64_t cap, uint32_t *__restrict__ tkey,
                                                   int32_t *__restrict__ tval)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    int32_t slot = 0;
    int cnt = 0;
    int64_t k0 = 0;
    if (r < n_splats) {
        slot = rank_ids[r];
        cnt = tiles[slot];
        k0 = offsets[r];
        if (k0 >= cap) cnt = 0;
    }
    int toff = 0, tx_n = 1;
    int4 b = make_int4(0, 0, 0, 0);
    if (cnt > 0) {
        const int c = camera_of_splat(cams, n_cams, slot);
        toff = cams[c].tile_offset;
        tx_n = cams[c].tiles_x;
        b = rect[slot];
    }
    if (cnt > 0 && cnt <= kEmitLaneMax) emit_tiles(k0, 0, 1, cnt, b, toff, tx_n, slot, cap, tkey, tval);
    // large boxes: the whole wave writes them, one splat at a time
    uint64_t big = __ballot(cnt > kEmitLaneMax);
    while (big) {
        const int src = __builtin_ctzll(big);
        big &= big - 1;
        const int bcnt = __shfl(cnt, src, kWave);
        const int64_t bk0 = __shfl(k0, src, kWave);
        const int32_t bslot = __shfl(slot, src, kWave);
        const int btoff = __shfl(toff, src, kWave), btx = __shfl(tx_n, src, kWave);
        const int4 bb = make_int4(__shfl(b.x, src, kWave), __shfl(b.y, src, kWave), __shfl(b.z, src, kWave),
                                  __shfl(b.w, src, kWave));
        emit_tiles(bk0, lane, kWave, bcnt, bb, btoff, btx, bslot, cap, tkey, tval);
    }
}

// -------------------------------------------------------------------------- ranges

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void ranges_kernel(const uint64_t *__restrict__ keys, const int64_t *__restrict__ counters,
                                                     int64_t cap, int32_t n_tiles, int32_t *__restrict__ ranges)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t kv = sort_count(counters, cap);
    if (k >= kv) return;
    const uint64_t t = keys[k] >> 32;
    if (t >= (uint64_t)n_tiles) return;
    if (k == 0 || (keys[k - 1] >> 32) != t) ranges[2 * t] = (int32_t)k;
    if (k == kv - 1 || (keys[k + 1] >> 32) != t) ranges[2 * t + 1] = (int32_t)(k + 1);
}

// ------------------------------------------------------------------------ work list

// Tiles with at least this many list entries are split into four quarter items.
constexpr int kSplitLen = 256;

__device__ inline int length_bucket(int len)
{
    // bucket 0 holds the longest lists; empty tiles land in the last bucket
    const int lg = 31 - __clz(len + 1);
    return kSchedNumBuckets - 1 - min(kSchedNumBuckets - 1, lg);
}

__global__ __launch_bounds__(64) void sched_clear_kernel(int32_t *__restrict__ sched)
{
    sched[threadIdx.x] = 0;
}

// Per-block bucket histogram in LDS, then one global atomic per non-empty bucket.
__global__ __launch_bounds__(256) void sched_count_kernel(const int32_t *__restrict__ ranges, int n_tiles,
                                                          int32_t *__restrict__ sched)
{
    __shared__ int cnt[kSchedNumBuckets];
    if (threadIdx.x < kSchedNumBuckets) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) {
        const int len = ranges[2 * t + 1] - ranges[2 * t];
        atomicAdd(&cnt[length_bucket(len)], len >= kSplitLen ? 4 : 1);
    }
    __syncthreads();
    if (threadIdx.x < kSchedNumBuckets && cnt[threadIdx.x])
        atomicAdd(&sched[kSchedBuckets + threadIdx.x], cnt[threadIdx.x]);
}

// Each block reserves one contiguous run per bucket (one global atomic per bucket), then
// hands out positions inside its runs with LDS atomics. Order inside a bucket is free.
__global__ __launch_bounds__(256) void sched_fill_kernel(const int32_t *__restrict__ ranges, int n_tiles,
                                                         int32_t *__restrict__ sched)
{
    __shared__ int cnt[kSchedNumBuckets], base[kSchedNumBuckets];
    if (threadIdx.x < kSchedNumBuckets) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int len = 0, b = 0, n = 0;
    if (t < n_tiles) {
        len = ranges[2 * t + 1] - ranges[2 * t];
        b = length_bucket(len);
        n = len >= kSplitLen ? 4 : 1;
        atomicAdd(&cnt[b], n);
    }
    __syncthreads();
    if (threadIdx.x < kSchedNumBuckets) {
        const int bk = threadIdx.x;
        int before = 0;
        for (int j = 0; j < bk; ++j) before += sched[kSchedBuckets + j];
        base[bk] = cnt[bk] ? before + atomicAdd(&sched[kSchedCursors + bk], cnt[bk]) : 0;
        cnt[bk] = 0;
        if (blockIdx.x == 0 && bk == 0) {
            int tot = 0;
            for (int j = 0; j < kSchedNumBuckets; ++j) tot += sched[kSchedBuckets + j];
            sched[kSchedItems] = tot;
        }
    }
    __syncthreads();
    if (t >= n_tiles) return;
    const int split = len >= kSplitLen;
    const int pos = base[b] + atomicAdd(&cnt[b], n);
    int32_t *items = sched + kSchedHeader;
    for (int part = 0; part < n; ++part) items[pos + part] = (t << 3) | (split << 2) | part;
}

// ------------------------------------------------------------------------ workspace

// Workspace: depth-sort buffers (two key/value pairs over P splats), per-rank emit offsets,
// scan partial sums, one 32-bit key/value pair over the capacity (the other pair of the
// tile-sort ping-pong lives in bins->keys / bins->ids until the last pass overwrites them),
// and the radix histogram table.
struct BinLayout {
    size_t dkeyA, dvalA, dkeyB, dvalB, dcount, offsets, scan_sums, tkey, tval, hist, hist_sums, total;
    int64_t depth_nb, tile_nb, hist_n;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static BinLayout bin_layout(int64_t n_splats, int64_t cap)
{
    BinLayout L{};
    L.depth_nb = (n_splats + kSortChunk - 1) / kSortChunk;
    L.tile_nb = (cap + kSortChunk - 1) / kSortChunk;
    L.hist_n = (L.depth_nb > L.tile_nb ? L.depth_nb : L.tile_nb) * kRadix;
    const size_t p4 = align256((size_t)n_splats * 4);
    size_t o = 0;
    L.dkeyA = o;     o += p4;
    L.dvalA = o;     o += p4;
    L.dkeyB = o;     o += p4;
    L.dvalB = o;     o += p4;
    L.dcount = o;    o += 256;
    L.offsets = o;   o += align256((size_t)n_splats * sizeof(int64_t));
    L.scan_sums = o; o += align256((size_t)(scan_blocks(n_splats) + 1) * sizeof(int64_t));
    L.tkey = o;      o += align256((size_t)cap * 4);
    L.tval = o;      o += align256((size_t)cap * 4);
    L.hist = o;      o += align256((size_t)L.hist_n * sizeof(unsigned));
    L.hist_sums = o; o += align256((size_t)(scan_blocks(L.hist_n) + 1) * sizeof(unsigned));
    L.total = o;
    return L;
}

static int tile_bits(int32_t n_tiles)
{
    int tb = 0;
    while ((1ll << tb) < (int64_t)n_tiles) ++tb;
    return tb;
}

// One stable LSD pass: histogram, scan of the digit-major table, scatter.
static int radix_pass(const uint32_t *kin, const int32_t *vin, const int64_t *count, int64_t cap, int shift,
                      int64_t nb, unsigned *hist, unsigned *hist_sums, uint32_t *kout, int32_t *vout,
                      uint64_t *keys64, const float *depth, hipStream_t st)
{
    if (nb == 0) return GS_OK;
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(kSortBlock), 0, st, kin, count, cap, shift,
                       (int)nb, hist);
    const int rc = scan_exclusive<unsigned, unsigned>(ArrayLoad<unsigned>{hist}, nb * kRadix, hist, hist_sums,
                                                      nullptr, nullptr, -1, st);
    if (rc != GS_OK) return rc;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kSortBlock), 0, st, kin, vin, count, cap,
                       shift, (int)nb, hist, kout, vout, keys64, depth);
    return check_launch("radix pass");
}

}  // namespace gsx

using namespace gsx;

static int build_schedule(gs_bins *bins, hipStream_t st)
{
    const unsigned g = grid_for(bins->n_tiles, 256);
    hipLaunchKernelGGL(sched_clear_kernel, dim3(1), dim3(kSchedHeader), 0, st, bins->schedule);
    hipLaunchKernelGGL(sched_count_kernel, dim3(g), dim3(256), 0, st, bins->ranges, bins->n_tiles, bins->schedule);
    hipLaunchKernelGGL(sched_fill_kernel, dim3(g), dim3(256), 0, st, bins->ranges, bins->n_tiles, bins->schedule);
    return check_launch("gs_bin_and_sort");
}

extern "C" int64_t gs_schedule_size(int32_t n_tiles)
{
    return n_tiles < 0 ? 0 : (int64_t)kSchedHeader + 4ll * n_tiles;
}

extern "C" size_t gs_bin_and_sort_workspace_size(int64_t n_splats, int64_t capacity, int32_t n_tiles)
{
    (void)n_tiles;
    if (n_splats < 0 || capacity < 1) return 0;
    return bin_layout(n_splats, capacity).total;
}

extern "C" int gs_bin_and_sort(const gs_splats *s, int64_t n_splats, const gs_camera *cams, int32_t n_cams,
                               gs_bins *bins, void *workspace, size_t workspace_bytes, void *stream)
{
    clear_error();
    if (!s || !cams || !bins || n_cams < 1 || n_splats < 0)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: null argument or bad size");
    if (bins->capacity < 1 || bins->capacity > 0x7fffffffll || bins->n_tiles < 1)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: capacity must be in [1, 2^31-1], n_tiles >= 1");
    if (n_splats > 0x7fffffffll)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: n_splats must be below 2^31");
    if (!bins->keys || !bins->ids || !bins->ranges || !bins->schedule || !bins->counters || !s->rect || !s->depth ||
        !s->tiles_touched || n_splats > s->capacity)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: null buffer or n_splats > capacity");
    const int64_t cap = bins->capacity;
    const BinLayout L = bin_layout(n_splats, cap);
    if (!workspace || workspace_bytes < L.total)
        return set_error(GS_ERR_CAPACITY, "gs_bin_and_sort: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    uint32_t *dkeyA = (uint32_t *)(ws + L.dkeyA), *dkeyB = (uint32_t *)(ws + L.dkeyB);
    int32_t *dvalA = (int32_t *)(ws + L.dvalA), *dvalB = (int32_t *)(ws + L.dvalB);
    int64_t *dcount = (int64_t *)(ws + L.dcount);
    int64_t *offsets = (int64_t *)(ws + L.offsets);
    int64_t *scan_sums = (int64_t *)(ws + L.scan_sums);
    unsigned *hist = (unsigned *)(ws + L.hist);
    unsigned *hist_sums = (unsigned *)(ws + L.hist_sums);
    const int64_t *K = (const int64_t *)bins->counters;

    // ranges start empty: (0, 0)
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(2ll * bins->n_tiles, 256)), dim3(256), 0, st, bins->ranges,
                       2ll * bins->n_tiles, 0);
    if (n_splats == 0) {
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(256), 0, st, (int32_t *)bins->counters, 4, 0);
        return build_schedule(bins, st);
    }

    // 1. depth order of the splats (four 8-bit passes: the result is back in A)
    hipLaunchKernelGGL(depth_keys_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, st, s->tiles_touched,
                       s->depth, n_splats, dkeyA, dvalA, dcount);
    int rc = GS_OK;
    for (int pass = 0; pass < 4 && rc == GS_OK; ++pass) {
        const bool even = (pass & 1) == 0;
        rc = radix_pass(even ? dkeyA : dkeyB, even ? dvalA : dvalB, dcount, n_splats, pass * kRadixBits, L.depth_nb,
                        hist, hist_sums, even ? dkeyB : dkeyA, even ? dvalB : dvalA, nullptr, nullptr, st);
    }
    if (rc != GS_OK) return rc;
    const int32_t *rank_ids = dvalA;

    // 2. emit offsets in depth-rank order; K and the overflow flag go to bins->counters
    rc = scan_exclusive<int64_t, int64_t>(RankTiles{s->tiles_touched, rank_ids}, n_splats, offsets, scan_sums,
                                          bins->counters, bins->counters + 1, cap, st);
    if (rc != GS_OK) return rc;

    // 3-4. emit, then stable passes by tile id. The last pass reads the workspace pair W and
    // writes bins; earlier passes alternate between W and the pair stored in bins' buffers.
    const int passes = max(1, (tile_bits(bins->n_tiles) + kRadixBits - 1) / kRadixBits);
    uint32_t *kW = (uint32_t *)(ws + L.tkey), *kX = (uint32_t *)bins->keys;
    int32_t *vW = (int32_t *)(ws + L.tval), *vX = bins->ids;
    const bool emit_to_W = ((passes - 1) & 1) == 0;
    uint32_t *kin = emit_to_W ? kW : kX;
    int32_t *vin = emit_to_W ? vW : vX;
    hipLaunchKernelGGL(emit_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, st, rank_ids, offsets,
                       s->tiles_touched, (const int4 *)s->rect, cams, (int)n_cams, n_splats, cap, kin, vin);
    rc = check_launch("emit");
    for (int pass = 0; pass < passes && rc == GS_OK; ++pass) {
        const bool last = pass == passes - 1;
        uint32_t *kout = kin == kW ? kX : kW;
        int32_t *vout = vin == vW ? vX : vW;
        rc = radix_pass(kin, vin, K, cap, pass * kRadixBits, L.tile_nb, hist, hist_sums, last ? nullptr : kout,
                        last ? bins->ids : vout, last ? bins->keys : nullptr, s->depth, st);
        kin = kout;
        vin = vout;
    }
    if (rc != GS_OK) return rc;

    // 5. tile ranges and the work list
    hipLaunchKernelGGL(ranges_kernel, dim3(grid_for(cap, 256)), dim3(256), 0, st, bins->keys, K, cap, bins->n_tiles,
                       bins->ranges);
    return build_schedule(bins, st);
}
