// gs_bin_and_sort: tile binning and per-tile depth order (Sec. 2.2).
//
//   1. exclusive scan of tiles_touched (int64) -> emit offsets, K = total
//   2. emit: each visible splat writes (global tile << 32 | depth bits, slot) for every
//      tile of its box, row-major, at its scan offset (entries beyond capacity are dropped
//      and the overflow flag is raised)
//   3. stable LSD radix sort over the low 32 + ceil(log2(n_tiles)) key bits; each pass is
//      a per-block digit histogram, a scan of the digit-major histogram table and a
//      stable scatter. Block ranking uses wave ballots to group equal digits and LDS
//      counters per (wave, digit), so no LDS atomics contend on popular digits.
//   4. ranges: [start, end) of each tile's run.
//
// Every kernel is sized from host-known capacities and reads K from device memory, so
// the whole sequence replays unchanged inside a captured HIP graph.
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

template <typename TIn, typename TAcc>
__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const TIn *__restrict__ in, int64_t n,
                                                                 TAcc *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    TAcc acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) acc += (TAcc)in[base + k];
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

template <typename TIn, typename TAcc, typename TOut>
__global__ __launch_bounds__(kScanBlock) void scan_down_kernel(const TIn *__restrict__ in, int64_t n,
                                                               const TAcc *__restrict__ sums,
                                                               TOut *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    TIn vals[kScanItems];
    TAcc acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = base + k < n ? in[base + k] : (TIn)0;
        acc += (TAcc)vals[k];
    }
    TAcc tot;
    TAcc run = block_exclusive_scan<TAcc>(acc, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = (TOut)run;
        run += (TAcc)vals[k];
    }
}

static int64_t scan_blocks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

// Exclusive scan of n values into out; sums needs scan_blocks(n) entries.
template <typename TIn, typename TAcc, typename TOut>
static int scan_exclusive(const TIn *in, int64_t n, TOut *out, TAcc *sums, int64_t *total, int64_t *flag,
                          int64_t cap, hipStream_t st)
{
    const int64_t nb = scan_blocks(n);
    if (nb == 0) return GS_OK;
    hipLaunchKernelGGL((scan_reduce_kernel<TIn, TAcc>), dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, sums);
    hipLaunchKernelGGL((scan_sums_kernel<TAcc>), dim3(1), dim3(kScanBlock), 0, st, sums, nb, total, flag, cap);
    hipLaunchKernelGGL((scan_down_kernel<TIn, TAcc, TOut>), dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n,
                       sums, out);
    return check_launch("scan");
}

// ------------------------------------------------------------------------------ emit

__global__ __launch_bounds__(256) void emit_kernel(const int32_t *__restrict__ tiles, const int64_t *__restrict__ offsets,
                                                   const int4 *__restrict__ rect, const float *__restrict__ depth,
                                                   const gs_camera *__restrict__ cams, int n_cams, int64_t n_splats,
                                                   int64_t cap, uint64_t *__restrict__ keys, int32_t *__restrict__ ids)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_splats) return;
    const int cnt = tiles[p];
    if (cnt <= 0) return;
    int64_t k = offsets[p];
    if (k >= cap) return;
    const int c = camera_of_splat(cams, n_cams, p);
    const int toff = cams[c].tile_offset, tx_n = cams[c].tiles_x;
    const int4 b = rect[p];
    const uint64_t dbits = (uint64_t)__float_as_uint(depth[p]);
    for (int ty = b.y; ty <= b.w; ++ty)
        for (int tx = b.x; tx <= b.z; ++tx) {
            if (k >= cap) return;
            const uint64_t tile = (uint64_t)(toff + ty * tx_n + tx);
            keys[k] = (tile << 32) | dbits;
            ids[k] = (int32_t)p;
            ++k;
        }
}

// ------------------------------------------------------------------------ radix sort

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kSortItems = 16;                       // keys per lane
constexpr int kSortChunk = kSortBlock * kSortItems;  // keys per block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

__device__ inline int64_t sort_count(const int64_t *counters, int64_t cap)
{
    const int64_t k = counters[0];
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
__device__ inline void count_digits(const uint64_t (&key)[kSortItems], int64_t chunk_base, int64_t kvalid,
                                    int shift, unsigned (*cnt)[kRadix])
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = chunk_base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        const bool ok = idx < kvalid;
        const uint64_t valid = __ballot(ok);
        if (valid == 0) break;
        const unsigned d = (unsigned)(key[r] >> shift) & (kRadix - 1);
        const uint64_t peers = match_digit(d, valid);
        if (ok && (peers & lanemask_lt()) == 0) cnt[wave][d] += (unsigned)__popcll(peers);
    }
}

__global__ __launch_bounds__(kSortBlock) void radix_hist_kernel(const uint64_t *__restrict__ keys,
                                                                const int64_t *__restrict__ counters, int64_t cap,
                                                                int shift, int nblocks, unsigned *__restrict__ hist)
{
    __shared__ unsigned cnt[kSortWaves][kRadix];
    for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortBlock) (&cnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t kvalid = sort_count(counters, cap);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base < kvalid) {
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        uint64_t key[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
            key[r] = idx < kvalid ? keys[idx] : 0ull;
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
// position of the first key with digit d in block b.
__global__ __launch_bounds__(kSortBlock) void radix_scatter_kernel(const uint64_t *__restrict__ keys_in,
                                                                   const int32_t *__restrict__ vals_in,
                                                                   const int64_t *__restrict__ counters, int64_t cap,
                                                                   int shift, int nblocks,
                                                                   const unsigned *__restrict__ hist_scan,
                                                                   uint64_t *__restrict__ keys_out,
                                                                   int32_t *__restrict__ vals_out)
{
    __shared__ unsigned cnt[kSortWaves][kRadix];
    const int64_t kvalid = sort_count(counters, cap);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base >= kvalid) return;   // uniform over the block
    for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortBlock) (&cnt[0][0])[d] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint64_t key[kSortItems];
    int32_t val[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        const bool ok = idx < kvalid;
        key[r] = ok ? keys_in[idx] : 0ull;
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
        const unsigned d = (unsigned)(key[r] >> shift) & (kRadix - 1);
        const uint64_t peers = match_digit(d, valid);
        const unsigned pos = cnt[wave][d] + (unsigned)__popcll(peers & lanemask_lt());
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & lanemask_lt()) == 0) cnt[wave][d] += (unsigned)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (ok) {
            keys_out[pos] = key[r];
            vals_out[pos] = val[r];
        }
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

struct BinLayout {
    size_t offsets, scan_sums, keys_alt, vals_alt, hist, hist_sums, total;
    int64_t scan_nb, sort_nb, hist_n;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static BinLayout bin_layout(int64_t n_splats, int64_t cap)
{
    BinLayout L{};
    L.scan_nb = scan_blocks(n_splats);
    L.sort_nb = (cap + kSortChunk - 1) / kSortChunk;
    L.hist_n = L.sort_nb * kRadix;
    size_t o = 0;
    L.offsets = o;   o += align256((size_t)n_splats * sizeof(int64_t));
    L.scan_sums = o; o += align256((size_t)(L.scan_nb + 1) * sizeof(int64_t));
    L.keys_alt = o;  o += align256((size_t)cap * sizeof(uint64_t));
    L.vals_alt = o;  o += align256((size_t)cap * sizeof(int32_t));
    L.hist = o;      o += align256((size_t)L.hist_n * sizeof(unsigned));
    L.hist_sums = o; o += align256((size_t)(scan_blocks(L.hist_n) + 1) * sizeof(unsigned));
    L.total = o;
    return L;
}

static int key_bits(int32_t n_tiles)
{
    int tb = 0;
    while ((1ll << tb) < (int64_t)n_tiles) ++tb;
    return 32 + tb;
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
    if (!bins->keys || !bins->ids || !bins->ranges || !bins->schedule || !bins->counters || !s->rect || !s->depth ||
        !s->tiles_touched || n_splats > s->capacity)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: null buffer or n_splats > capacity");
    const int64_t cap = bins->capacity;
    const BinLayout L = bin_layout(n_splats, cap);
    if (!workspace || workspace_bytes < L.total)
        return set_error(GS_ERR_CAPACITY, "gs_bin_and_sort: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int64_t *offsets = (int64_t *)(ws + L.offsets);
    int64_t *scan_sums = (int64_t *)(ws + L.scan_sums);
    uint64_t *keys_alt = (uint64_t *)(ws + L.keys_alt);
    int32_t *vals_alt = (int32_t *)(ws + L.vals_alt);
    unsigned *hist = (unsigned *)(ws + L.hist);
    unsigned *hist_sums = (unsigned *)(ws + L.hist_sums);

    // ranges start empty: (0, 0)
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(2ll * bins->n_tiles, 256)), dim3(256), 0, st, bins->ranges,
                       2ll * bins->n_tiles, 0);
    if (n_splats == 0) {
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(256), 0, st, (int32_t *)bins->counters, 4, 0);
        return build_schedule(bins, st);
    }
    int rc = scan_exclusive<int32_t, int64_t, int64_t>(s->tiles_touched, n_splats, offsets, scan_sums,
                                                        bins->counters, bins->counters + 1, cap, st);
    if (rc != GS_OK) return rc;

    const int passes = (key_bits(bins->n_tiles) + kRadixBits - 1) / kRadixBits;
    // emit into the buffer that makes the last pass land in bins->keys / bins->ids
    uint64_t *kA = (passes % 2 == 0) ? bins->keys : keys_alt;
    int32_t *vA = (passes % 2 == 0) ? bins->ids : vals_alt;
    uint64_t *kB = (passes % 2 == 0) ? keys_alt : bins->keys;
    int32_t *vB = (passes % 2 == 0) ? vals_alt : bins->ids;
    hipLaunchKernelGGL(emit_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, st, s->tiles_touched, offsets,
                       (const int4 *)s->rect, s->depth, cams, (int)n_cams, n_splats, cap, kA, vA);
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * kRadixBits;
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)L.sort_nb), dim3(kSortBlock), 0, st, kA,
                           (const int64_t *)bins->counters, cap, shift, (int)L.sort_nb, hist);
        rc = scan_exclusive<unsigned, unsigned, unsigned>(hist, L.hist_n, hist, hist_sums, nullptr, nullptr, -1, st);
        if (rc != GS_OK) return rc;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)L.sort_nb), dim3(kSortBlock), 0, st, kA, vA,
                           (const int64_t *)bins->counters, cap, shift, (int)L.sort_nb, hist, kB, vB);
        uint64_t *tk = kA; kA = kB; kB = tk;
        int32_t *tv = vA; vA = vB; vB = tv;
    }
    hipLaunchKernelGGL(ranges_kernel, dim3(grid_for(cap, 256)), dim3(256), 0, st, bins->keys,
                       (const int64_t *)bins->counters, cap, bins->n_tiles, bins->ranges);
    return build_schedule(bins, st);
}
