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
// Each pass is one launch of a single-pass LSD sort with decoupled look-back: one upfront
// kernel counts the digits of all passes from one read of the keys; then, per pass, each
// block ranks its chunk, publishes its digit counts, sums its predecessors' published
// counts for its global offsets (waiting, with a spin limit, on any predecessor that has
// not published yet), stages the chunk in LDS in digit order and writes it out in runs.
// Block ranking uses wave ballots to group equal digits and LDS counters per (wave,
// digit), so no LDS atomics contend on popular digits. Every kernel is sized from
// host-known capacities and reads its element count from device memory, and the
// look-back state is cleared by a kernel at the start of each call, so the whole sequence
// replays unchanged inside a captured HIP graph.
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
constexpr int kMaxTilePassesDev = 4;   // tile ids are int32: at most four 8-bit passes
static_assert(kSortBlock == kRadix, "one thread per digit in the single-pass sort");

__device__ inline int64_t sort_count(const int64_t *counter, int64_t cap)
{
    const int64_t k = *counter;
    return k < cap ? k : cap;
}

// Entries the tile passes sort: all K of them, or none when K exceeds the capacity (the
// list is then not built at all: every range is empty and the caller regrows).
__device__ inline int64_t tile_sort_count(const int64_t *counter, int64_t cap)
{
    const int64_t k = *counter;
    return k <= cap ? k : 0;
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

// Digit histograms of every pass from one read of the keys: ghist[pass][digit].
__global__ __launch_bounds__(kSortBlock) void radix_global_hist_kernel(const uint32_t *__restrict__ keys,
                                                                       const int64_t *__restrict__ count, int64_t cap,
                                                                       int passes, unsigned *__restrict__ ghist)
{
    __shared__ unsigned cnt[kSortWaves][kRadix];
    const int64_t kvalid = sort_count(count, cap);
    const int64_t base = (int64_t)blockIdx.x * kSortChunk;
    if (base >= kvalid) return;   // uniform over the block
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t key[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        key[r] = idx < kvalid ? keys[idx] : 0u;
    }
    for (int pass = 0; pass < passes; ++pass) {
        for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortBlock) (&cnt[0][0])[d] = 0;
        __syncthreads();
        count_digits(key, base, kvalid, pass * kRadixBits, cnt);
        __syncthreads();
        const int d = threadIdx.x;   // kSortBlock == kRadix
        unsigned tot = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) tot += cnt[w][d];
        if (tot) atomicAdd(&ghist[pass * kRadix + d], tot);
        __syncthreads();
    }
}

// Status word of one (block, digit) in a single-pass sort: 0 = not yet published,
// kStatAgg | count of the block's own keys, kStatInc | inclusive prefix (global position
// one past the block's last key with that digit).
constexpr uint64_t kStatAgg = 1ull << 62;
constexpr uint64_t kStatInc = 2ull << 62;
constexpr uint64_t kStatValue = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 24;   // bounded wait: a predecessor that never publishes ends the wait

// LDS of one single-pass sort block.
struct SweepShared {
    unsigned cnt[kSortWaves][kRadix];   // per-(wave, digit) counts, then staging cursors
    unsigned lstart[kRadix];            // staging start of each digit
    int64_t gbase[kRadix];              // global position of the block's first key per digit
    uint32_t skey[kSortChunk];          // staged keys (digit order); first holds rank offsets
    int32_t sval[kSortChunk];
    int chunk, gave_up;
};

__device__ inline int sweep_ticket(SweepShared &sh, int32_t *ticket)
{
    if (threadIdx.x == 0) {
        sh.chunk = atomicAdd(ticket, 1);
        sh.gave_up = 0;
    }
    for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortBlock) (&sh.cnt[0][0])[d] = 0;
    __syncthreads();
    return sh.chunk;
}

// One stable LSD pass over chunk b, keys already in registers in the wave-strided layout
// (lane l of wave w holds, in row r, key base + w * kSortChunk / kSortWaves + 64 r + l).
// The block ranks its chunk (wave ballots, per-(wave, digit) LDS counters), publishes its
// digit counts, looks back over its predecessors' published counts for its global
// offsets, stages the chunk in LDS in digit order and writes it out in runs. With
// keys64_out set (the last tile pass) it writes ids and the 64-bit keys
// (tile << 32 | depth bits of the value) instead of 32-bit keys.
__device__ inline void sweep_body(SweepShared &sh, const uint32_t (&key)[kSortItems],
                                  const int32_t (&val)[kSortItems], int b, int64_t base, int64_t kvalid, int shift,
                                  const unsigned *__restrict__ ghist, uint64_t *__restrict__ status,
                                  uint32_t *__restrict__ keys_out, int32_t *__restrict__ vals_out,
                                  uint64_t *__restrict__ keys64_out, const float *__restrict__ depth,
                                  int64_t n_splats, int64_t *__restrict__ err_flag)
{
    const int n_here = (int)min((int64_t)kSortChunk, kvalid - base);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    count_digits(key, base, kvalid, shift, sh.cnt);
    __syncthreads();

    // thread d owns digit d
    const int d = threadIdx.x;
    unsigned tot = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) tot += sh.cnt[w][d];
    int64_t gtot;
    const int64_t dstart = block_exclusive_scan<int64_t>((int64_t)ghist[d], &gtot);   // first slot of digit d
    uint64_t *my = status + (int64_t)b * kRadix + d;
    int64_t excl = dstart;
    if (b == 0) {
        __hip_atomic_store(my, kStatInc | (uint64_t)(dstart + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(my, kStatAgg | (uint64_t)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t acc = 0;
        int j = b - 1;
        int spins = 0;
        while (true) {
            const uint64_t st = __hip_atomic_load(status + (int64_t)j * kRadix + d, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t flag = st & ~kStatValue;
            if (flag == 0) {
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    sh.gave_up = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            acc += (int64_t)(st & kStatValue);
            if (flag == kStatInc) break;
            --j;
        }
        excl = acc;
        __hip_atomic_store(my, kStatInc | (uint64_t)(acc + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    sh.gbase[d] = excl;
    unsigned ltot;
    const unsigned ls = block_exclusive_scan<unsigned>(tot, &ltot);
    sh.lstart[d] = ls;
    // per-(wave, digit) cursors into the staging buffer
    unsigned run = ls;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
        const unsigned c = sh.cnt[w][d];
        sh.cnt[w][d] = run;
        run += c;
    }
    __syncthreads();
    if (sh.gave_up) return;   // offsets unknown: write nothing (the error word is set)

    // stage the chunk in digit order (stable: waves in order, lanes in order within a wave)
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        const bool ok = idx < kvalid;
        const uint64_t valid = __ballot(ok);
        if (valid == 0) break;
        const unsigned dg = (key[r] >> shift) & (kRadix - 1);
        const uint64_t peers = match_digit(dg, valid);
        const unsigned pos = sh.cnt[wave][dg] + (unsigned)__popcll(peers & lanemask_lt());
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & lanemask_lt()) == 0) sh.cnt[wave][dg] += (unsigned)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (ok) {
            sh.skey[pos] = key[r];
            sh.sval[pos] = val[r];
        }
    }
    __syncthreads();

    // write out: consecutive threads take consecutive staged keys, so each digit's run of
    // this chunk is written by consecutive lanes to consecutive addresses
    for (int i = threadIdx.x; i < n_here; i += kSortBlock) {
        const uint32_t k = sh.skey[i];
        const int32_t v = sh.sval[i];
        const unsigned dg = (k >> shift) & (kRadix - 1);
        const int64_t g = sh.gbase[dg] + (i - (int)sh.lstart[dg]);
        if (g < 0 || g >= kvalid) continue;   // unreachable when the counts are consistent
        vals_out[g] = v;
        if (keys64_out) {
            // v is a splat slot by construction; the test keeps a broken invariant from
            // turning into a wild read
            const uint32_t dbits = (uint64_t)(uint32_t)v < (uint64_t)n_splats ? __float_as_uint(depth[v]) : 0u;
            keys64_out[g] = ((uint64_t)k << 32) | (uint64_t)dbits;
        } else {
            keys_out[g] = k;
        }
    }
}

// One stable LSD pass with decoupled look-back (chained scan over blocks), in one launch.
// Blocks take chunk indices from a ticket counter in launch order, so every chunk a block
// waits on belongs to a block that is already running.
__global__ __launch_bounds__(kSortBlock) void onesweep_kernel(const uint32_t *__restrict__ keys_in,
                                                              const int32_t *__restrict__ vals_in,
                                                              const int64_t *__restrict__ count, int64_t cap,
                                                              int shift, const unsigned *__restrict__ ghist,
                                                              uint64_t *__restrict__ status,
                                                              int32_t *__restrict__ ticket,
                                                              uint32_t *__restrict__ keys_out,
                                                              int32_t *__restrict__ vals_out,
                                                              uint64_t *__restrict__ keys64_out,
                                                              const float *__restrict__ depth,
                                                              int64_t n_splats, int all_or_none,
                                                              int64_t *__restrict__ err_flag)
{
    __shared__ SweepShared sh;
    const int b = sweep_ticket(sh, ticket);
    const int64_t kvalid = all_or_none ? tile_sort_count(count, cap) : sort_count(count, cap);
    const int64_t base = (int64_t)b * kSortChunk;
    if (base >= kvalid) return;   // uniform over the block; no valid chunk waits on it
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
    sweep_body(sh, key, val, b, base, kvalid, shift, ghist, status, keys_out, vals_out, keys64_out, depth, n_splats,
               err_flag);
}

// The first tile pass, over entries it generates itself: list entry k belongs to the splat
// of depth rank r with offsets[r] <= k < offsets[r] + tiles, as its (k - offsets[r])-th box
// tile in row-major order; its key is the global tile id and its value the splat slot. The
// block reads the rank offsets of its chunk into LDS, each thread generates 16 consecutive
// entries (one search for the first, then walking the box), and the chunk is regrouped
// into the strided layout of the ranking.
__global__ __launch_bounds__(kSortBlock) void onesweep_emit_kernel(
    const int32_t *__restrict__ rank_ids, const int64_t *__restrict__ offsets, const int32_t *__restrict__ chunk_rank,
    const int32_t *__restrict__ tiles, const int4 *__restrict__ rect, const gs_camera *__restrict__ cams, int n_cams,
    int64_t n_splats, const int64_t *__restrict__ count, int64_t cap, const unsigned *__restrict__ ghist,
    uint64_t *__restrict__ status, int32_t *__restrict__ ticket, uint32_t *__restrict__ keys_out,
    int32_t *__restrict__ vals_out, uint64_t *__restrict__ keys64_out, const float *__restrict__ depth,
    int64_t *__restrict__ err_flag)
{
    __shared__ SweepShared sh;
    __shared__ int n_ranks;
    const int b = sweep_ticket(sh, ticket);
    const int64_t kvalid = tile_sort_count(count, cap);
    const int64_t base = (int64_t)b * kSortChunk;
    if (base >= kvalid) return;   // uniform over the block
    const int n_here = (int)min((int64_t)kSortChunk, kvalid - base);
    const int64_t n_chunks = (kvalid + kSortChunk - 1) / kSortChunk;
    const int r0 = chunk_rank[b];
    if (threadIdx.x == 0) {
        const int64_t r_end = b + 1 < n_chunks ? (int64_t)chunk_rank[b + 1] : n_splats - 1;
        n_ranks = (int)min((int64_t)kSortChunk, r_end - r0 + 1);
        // a rank outside [0, n_splats) would mean inconsistent counts: report, write nothing
        if (r0 < 0 || r0 >= n_splats || r_end < r0 || r_end >= n_splats) {
            n_ranks = 0;
            __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    const int nr = n_ranks;
    if (nr == 0) return;   // uniform; successors waiting on this chunk give up after the spin limit
    // rank start offsets relative to the chunk (the first one is <= 0)
    int32_t *roff = (int32_t *)sh.skey;
    for (int i = threadIdx.x; i < nr; i += kSortBlock) roff[i] = (int32_t)(offsets[r0 + i] - base);
    __syncthreads();

    uint32_t gk[kSortItems];
    int32_t gv[kSortItems];
    const int e0 = threadIdx.x * kSortItems;   // chunk-relative index of this thread's first entry
    if (e0 < n_here) {
        int lo = 0, hi = nr - 1;               // last rank with roff <= e0
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (roff[mid] <= e0) lo = mid; else hi = mid - 1;
        }
        int ri = lo;
        int slot = rank_ids[r0 + ri];
        int4 bx = rect[slot];
        int c = camera_of_splat(cams, n_cams, slot);
        int toff = cams[c].tile_offset, tx_n = cams[c].tiles_x;
        int w = bx.z - bx.x + 1;
        int j = e0 - roff[ri];                 // index within the splat's box
        int ntile = tiles[slot];
        int ty = bx.y + j / w, tx = bx.x + j % w;
#pragma unroll
        for (int q = 0; q < kSortItems; ++q) {
            if (j == ntile && e0 + q < n_here) {  // next splat in rank order
                ++ri;
                slot = rank_ids[r0 + ri];
                bx = rect[slot];
                c = camera_of_splat(cams, n_cams, slot);
                toff = cams[c].tile_offset;
                tx_n = cams[c].tiles_x;
                w = bx.z - bx.x + 1;
                ntile = tiles[slot];
                j = 0;
                ty = bx.y;
                tx = bx.x;
            }
            gk[q] = (uint32_t)(toff + ty * tx_n + tx);
            gv[q] = slot;
            ++j;
            if (++tx > bx.z) {
                tx = bx.x;
                ++ty;
            }
        }
    }
    __syncthreads();   // roff is no longer read
    if (e0 < n_here) {
#pragma unroll
        for (int q = 0; q < kSortItems; ++q) {
            sh.skey[e0 + q] = gk[q];
            sh.sval[e0 + q] = gv[q];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t key[kSortItems];
    int32_t val[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int i = wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        const bool ok = i < n_here;
        key[r] = ok ? sh.skey[i] : 0u;
        val[r] = ok ? sh.sval[i] : 0;
    }
    __syncthreads();   // the staging arrays are reused by the ranking
    sweep_body(sh, key, val, b, base, kvalid, 0, ghist, status, keys_out, vals_out, keys64_out, depth, n_splats,
               err_flag);
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

// ----------------------------------------------------------- tile-pass histograms, emit

// Digit histograms of all tile passes, counted from the boxes without emitting anything:
// a box row covers the consecutive global tile ids [a, a + L). For the lowest digit those
// are L consecutive values mod 256 (L / 256 full turns plus a cyclic run, added to a
// difference array); for a higher digit of weight 256^p the row splits into at most
// L / 256^p + 2 runs of equal digit. A fixed grid of blocks strides over the splats and
// adds its LDS histograms to the global ones once. Nothing is counted when K exceeds the
// capacity (the list is then not built).
constexpr int kHistBlocks = 1024;

__global__ __launch_bounds__(256) void tile_hist_kernel(const int32_t *__restrict__ tiles,
                                                        const int4 *__restrict__ rect,
                                                        const gs_camera *__restrict__ cams, int n_cams,
                                                        int64_t n_splats, const int64_t *__restrict__ K, int64_t cap,
                                                        int passes, unsigned *__restrict__ ghist)
{
    __shared__ int diff0[kRadix + 1];
    __shared__ unsigned full0;
    __shared__ unsigned h[kMaxTilePassesDev][kRadix];
    for (int i = threadIdx.x; i < kRadix + 1; i += blockDim.x) diff0[i] = 0;
    for (int i = threadIdx.x; i < kMaxTilePassesDev * kRadix; i += blockDim.x) (&h[0][0])[i] = 0;
    if (threadIdx.x == 0) full0 = 0;
    __syncthreads();
    if (*K > cap) return;   // uniform: every thread reads the same K
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_splats;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (tiles[p] <= 0) continue;
        const int c = camera_of_splat(cams, n_cams, p);
        const int toff = cams[c].tile_offset, TX = cams[c].tiles_x;
        const int4 bx = rect[p];
        const int L = bx.z - bx.x + 1;
        for (int y = bx.y; y <= bx.w; ++y) {
            const int64_t a = (int64_t)toff + (int64_t)y * TX + bx.x, e = a + L - 1;
            const int s0 = (int)(a & (kRadix - 1)), r = L & (kRadix - 1);
            if (L >> kRadixBits) atomicAdd(&full0, (unsigned)(L >> kRadixBits));
            if (r) {
                atomicAdd(&diff0[s0], 1);
                if (s0 + r <= kRadix) {
                    atomicAdd(&diff0[s0 + r], -1);
                } else {
                    atomicAdd(&diff0[0], 1);
                    atomicAdd(&diff0[s0 + r - kRadix], -1);
                }
            }
            for (int pass = 1; pass < passes; ++pass) {
                const int sh = pass * kRadixBits;
                for (int64_t blk = a >> sh; blk <= (e >> sh); ++blk) {
                    const int64_t lo = max(a, blk << sh), hi = min(e, ((blk + 1) << sh) - 1);
                    atomicAdd(&h[pass][blk & (kRadix - 1)], (unsigned)(hi - lo + 1));
                }
            }
        }
    }
    __syncthreads();
    const int d = threadIdx.x;   // blockDim.x == kRadix
    int tot;
    const int run = block_exclusive_scan<int>(diff0[d], &tot) + diff0[d];
    const unsigned v0 = full0 + (unsigned)run;
    if (v0) atomicAdd(&ghist[d], v0);
    for (int pass = 1; pass < passes; ++pass)
        if (h[pass][d]) atomicAdd(&ghist[pass * kRadix + d], h[pass][d]);
}

// Splats whose box has at most this many tiles are emitted by their own lane.
constexpr int kEmitLaneMax = 16;

__device__ inline void emit_tiles(int64_t k0, int count_begin, int count_step, int n_tiles_box, const int4 &b,
                                  int toff, int tx_n, int32_t slot, uint32_t *__restrict__ tkey,
                                  int32_t *__restrict__ tval)
{
    const int w = b.z - b.x + 1;
    for (int j = count_begin; j < n_tiles_box; j += count_step) {
        const int64_t k = k0 + j;
        const int ty = b.y + j / w, tx = b.x + j % w;
        tkey[k] = (uint32_t)(toff + ty * tx_n + tx);
        tval[k] = slot;
    }
}

// Emit in depth-rank order, one thread per rank: (global tile id, slot) for every tile of
// the box, row-major, at the rank's offset. Nothing is written when K exceeds the capacity.
__global__ __launch_bounds__(256) void emit_kernel(const int32_t *__restrict__ rank_ids,
                                                   const int64_t *__restrict__ offsets,
                                                   const int32_t *__restrict__ tiles, const int4 *__restrict__ rect,
                                                   const gs_camera *__restrict__ cams, int n_cams, int64_t n_splats,
                                                   const int64_t *__restrict__ K, int64_t cap,
                                                   uint32_t *__restrict__ tkey, int32_t *__restrict__ tval)
{
    if (*K > cap) return;   // uniform
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    int32_t slot = 0;
    int cnt = 0;
    int64_t k0 = 0;
    if (r < n_splats) {
        slot = rank_ids[r];
        cnt = tiles[slot];
        k0 = offsets[r];
    }
    int toff = 0, tx_n = 1;
    int4 b = make_int4(0, 0, 0, 0);
    if (cnt > 0) {
        const int c = camera_of_splat(cams, n_cams, slot);
        toff = cams[c].tile_offset;
        tx_n = cams[c].tiles_x;
        b = rect[slot];
    }
    if (cnt > 0 && cnt <= kEmitLaneMax) emit_tiles(k0, 0, 1, cnt, b, toff, tx_n, slot, tkey, tval);
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
        emit_tiles(bk0, lane, kWave, bcnt, bb, btoff, btx, bslot, tkey, tval);
    }
}

// [start, end) of each tile's run in the sorted list (nothing when the list was not built).
__global__ __launch_bounds__(256) void ranges_kernel(const uint64_t *__restrict__ keys,
                                                     const int64_t *__restrict__ K, int64_t cap, int32_t n_tiles,
                                                     int32_t *__restrict__ ranges)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t kv = tile_sort_count(K, cap);
    if (k >= kv) return;
    const uint64_t t = keys[k] >> 32;
    if (t >= (uint64_t)n_tiles) return;
    if (k == 0 || (keys[k - 1] >> 32) != t) ranges[2 * t] = (int32_t)k;
    if (k == kv - 1 || (keys[k + 1] >> 32) != t) ranges[2 * t + 1] = (int32_t)(k + 1);
}

// Folds the sort's error word into the overflow flag (value 2: a look-back wait gave up).
__global__ __launch_bounds__(64) void err_fold_kernel(int64_t *__restrict__ counters, const int64_t *__restrict__ err)
{
    if (threadIdx.x == 0 && *err) counters[1] |= *err;
}

// chunk_rank[c] = depth rank of the splat that holds list entry c * kSortChunk.
__global__ __launch_bounds__(256) void chunk_rank_kernel(const int32_t *__restrict__ rank_ids,
                                                         const int64_t *__restrict__ offsets,
                                                         const int32_t *__restrict__ tiles, int64_t n_splats,
                                                         const int64_t *__restrict__ count, int64_t cap,
                                                         int32_t *__restrict__ chunk_rank)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_splats) return;
    const int n = tiles[rank_ids[r]];
    if (n <= 0) return;
    const int64_t kvalid = tile_sort_count(count, cap);
    const int64_t s = offsets[r], e = s + n;
    for (int64_t c = (s + kSortChunk - 1) / kSortChunk; c * kSortChunk < e && c * kSortChunk < kvalid; ++c)
        chunk_rank[c] = (int32_t)r;
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------------ work list

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
                                                          int split_len, int split_parts, int32_t *__restrict__ sched)
{
    __shared__ int cnt[kSchedNumBuckets];
    if (threadIdx.x < kSchedNumBuckets) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) {
        const int len = ranges[2 * t + 1] - ranges[2 * t];
        atomicAdd(&cnt[length_bucket(len)], len >= split_len ? split_parts : 1);
    }
    __syncthreads();
    if (threadIdx.x < kSchedNumBuckets && cnt[threadIdx.x])
        atomicAdd(&sched[kSchedBuckets + threadIdx.x], cnt[threadIdx.x]);
}

// Each block reserves one contiguous run per bucket (one global atomic per bucket), then
// hands out positions inside its runs with LDS atomics. Order inside a bucket is free.
__global__ __launch_bounds__(256) void sched_fill_kernel(const int32_t *__restrict__ ranges, int n_tiles,
                                                         int split_len, int split_parts, int32_t *__restrict__ sched)
{
    __shared__ int cnt[kSchedNumBuckets], base[kSchedNumBuckets];
    if (threadIdx.x < kSchedNumBuckets) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int len = 0, b = 0, n = 0;
    if (t < n_tiles) {
        len = ranges[2 * t + 1] - ranges[2 * t];
        b = length_bucket(len);
        n = len >= split_len ? split_parts : 1;
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
            sched[kSchedParts] = split_parts;
        }
    }
    __syncthreads();
    if (t >= n_tiles) return;
    const int split = len >= split_len;
    const int pos = base[b] + atomicAdd(&cnt[b], n);
    int32_t *items = sched + kSchedHeader;
    for (int part = 0; part < n; ++part) items[pos + part] = (t << 3) | (split << 2) | part;
}

// ------------------------------------------------------------------------ workspace

// Workspace: depth-sort buffers (two key/value pairs over P splats), per-rank emit offsets,
// scan partial sums, one 32-bit key/value pair over the capacity (the other pair of the
// tile-sort ping-pong lives in bins->keys / bins->ids until the last pass overwrites them),
// then a region cleared at the start of every call: the look-back status words of every
// pass, the digit histograms, the chunk tickets and an error word.
constexpr int kDepthPasses = 4;
constexpr int kMaxTilePasses = 4;

struct BinLayout {
    size_t dkeyA, dvalA, dkeyB, dvalB, dcount, offsets, scan_sums, tkey, tval, chunk_rank;
    size_t zero_begin, stat_depth, stat_tile, ghist_depth, ghist_tile, tickets, err, total;
    int64_t depth_nb, tile_nb;
    int tile_passes;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int tile_bits(int32_t n_tiles)
{
    int tb = 0;
    while ((1ll << tb) < (int64_t)n_tiles) ++tb;
    return tb;
}

static int tile_passes_for(int32_t n_tiles)
{
    return max(1, (tile_bits(n_tiles) + kRadixBits - 1) / kRadixBits);
}

static BinLayout bin_layout(int64_t n_splats, int64_t cap, int32_t n_tiles)
{
    BinLayout L{};
    L.depth_nb = (n_splats + kSortChunk - 1) / kSortChunk;
    L.tile_nb = (cap + kSortChunk - 1) / kSortChunk;
    L.tile_passes = tile_passes_for(n_tiles);
    const size_t p4 = align256((size_t)n_splats * 4);
    const size_t stat_row = (size_t)kRadix * sizeof(uint64_t);
    size_t o = 0;
    L.dkeyA = o;       o += p4;
    L.dvalA = o;       o += p4;
    L.dkeyB = o;       o += p4;
    L.dvalB = o;       o += p4;
    L.dcount = o;      o += 256;
    L.offsets = o;     o += align256((size_t)n_splats * sizeof(int64_t));
    L.scan_sums = o;   o += align256((size_t)(scan_blocks(n_splats) + 1) * sizeof(int64_t));
    L.tkey = o;        o += align256((size_t)cap * 4);
    L.tval = o;        o += align256((size_t)cap * 4);
    L.chunk_rank = o;  o += align256((size_t)(L.tile_nb + 1) * sizeof(int32_t));
    L.zero_begin = o;
    L.stat_depth = o;  o += align256((size_t)kDepthPasses * L.depth_nb * stat_row);
    L.stat_tile = o;   o += align256((size_t)L.tile_passes * L.tile_nb * stat_row);
    L.ghist_depth = o; o += align256((size_t)kDepthPasses * kRadix * sizeof(unsigned));
    L.ghist_tile = o;  o += align256((size_t)kMaxTilePasses * kRadix * sizeof(unsigned));
    L.tickets = o;     o += 256;
    L.err = o;         o += 256;
    L.total = o;
    return L;
}

}  // namespace gsx

using namespace gsx;

static int build_schedule(gs_bins *bins, hipStream_t st)
{
    const unsigned g = grid_for(bins->n_tiles, 256);
    hipLaunchKernelGGL(sched_clear_kernel, dim3(1), dim3(kSchedHeader), 0, st, bins->schedule);
    const gs_tuning &tu = current_tuning();
    hipLaunchKernelGGL(sched_count_kernel, dim3(g), dim3(256), 0, st, bins->ranges, bins->n_tiles, tu.split_len,
                       tu.split_parts, bins->schedule);
    hipLaunchKernelGGL(sched_fill_kernel, dim3(g), dim3(256), 0, st, bins->ranges, bins->n_tiles, tu.split_len,
                       tu.split_parts, bins->schedule);
    return check_launch("gs_bin_and_sort");
}

extern "C" int64_t gs_schedule_size(int32_t n_tiles)
{
    return n_tiles < 0 ? 0 : (int64_t)kSchedHeader + 4ll * n_tiles;
}

extern "C" size_t gs_bin_and_sort_workspace_size(int64_t n_splats, int64_t capacity, int32_t n_tiles)
{
    if (n_splats < 0 || capacity < 1 || n_tiles < 1) return 0;
    return bin_layout(n_splats, capacity, n_tiles).total;
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
    const BinLayout L = bin_layout(n_splats, cap, bins->n_tiles);
    if (!workspace || workspace_bytes < L.total)
        return set_error(GS_ERR_CAPACITY, "gs_bin_and_sort: workspace too small");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    uint32_t *dkeyA = (uint32_t *)(ws + L.dkeyA), *dkeyB = (uint32_t *)(ws + L.dkeyB);
    int32_t *dvalA = (int32_t *)(ws + L.dvalA), *dvalB = (int32_t *)(ws + L.dvalB);
    int64_t *dcount = (int64_t *)(ws + L.dcount);
    int64_t *offsets = (int64_t *)(ws + L.offsets);
    int64_t *scan_sums = (int64_t *)(ws + L.scan_sums);
    uint64_t *stat_depth = (uint64_t *)(ws + L.stat_depth), *stat_tile = (uint64_t *)(ws + L.stat_tile);
    unsigned *ghist_depth = (unsigned *)(ws + L.ghist_depth), *ghist_tile = (unsigned *)(ws + L.ghist_tile);
    int32_t *tickets = (int32_t *)(ws + L.tickets);
    int64_t *err = (int64_t *)(ws + L.err);
    const int64_t *K = (const int64_t *)bins->counters;

    // ranges start empty: (0, 0)
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(2ll * bins->n_tiles, 256)), dim3(256), 0, st, bins->ranges,
                       2ll * bins->n_tiles, 0);
    if (n_splats == 0) {
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(256), 0, st, (int32_t *)bins->counters, 4, 0);
        return build_schedule(bins, st);
    }
    int rc = gs_zero(ws + L.zero_begin, L.total - L.zero_begin, st);
    if (rc != GS_OK) return rc;

    // 1. depth order of the splats (four 8-bit passes: the result is back in A)
    hipLaunchKernelGGL(depth_keys_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, st, s->tiles_touched,
                       s->depth, n_splats, dkeyA, dvalA, dcount);
    hipLaunchKernelGGL(radix_global_hist_kernel, dim3((unsigned)L.depth_nb), dim3(kSortBlock), 0, st, dkeyA,
                       (const int64_t *)dcount, n_splats, kDepthPasses, ghist_depth);
    for (int pass = 0; pass < kDepthPasses; ++pass) {
        const bool even = (pass & 1) == 0;
        hipLaunchKernelGGL(onesweep_kernel, dim3((unsigned)L.depth_nb), dim3(kSortBlock), 0, st,
                           even ? dkeyA : dkeyB, even ? dvalA : dvalB, (const int64_t *)dcount, n_splats,
                           pass * kRadixBits, ghist_depth + pass * kRadix,
                           stat_depth + (int64_t)pass * L.depth_nb * kRadix, tickets + pass, even ? dkeyB : dkeyA,
                           even ? dvalB : dvalA, (uint64_t *)nullptr, (const float *)nullptr, n_splats, 0, err);
    }
    rc = check_launch("depth sort");
    if (rc != GS_OK) return rc;
    const int32_t *rank_ids = dvalA;

    // 2. emit offsets in depth-rank order; K and the overflow flag go to bins->counters
    rc = scan_exclusive<int64_t, int64_t>(RankTiles{s->tiles_touched, rank_ids}, n_splats, offsets, scan_sums,
                                          bins->counters, bins->counters + 1, cap, st);
    if (rc != GS_OK) return rc;

    // 3. digit histograms of the tile passes, from the boxes
    const int passes = L.tile_passes;
    hipLaunchKernelGGL(tile_hist_kernel, dim3(kHistBlocks), dim3(256), 0, st, s->tiles_touched, (const int4 *)s->rect,
                       cams, (int)n_cams, n_splats, K, cap, passes, ghist_tile);

    // 4. stable passes by tile id. The first pass takes the entries in depth-rank order,
    // either emitted into a buffer or generated inside the pass (launch tuning); the last
    // reads the workspace pair W and writes bins; in between, passes alternate between W
    // and the pair stored in bins' buffers.
    uint32_t *kW = (uint32_t *)(ws + L.tkey), *kX = (uint32_t *)bins->keys;
    int32_t *vW = (int32_t *)(ws + L.tval), *vX = bins->ids;
    // the buffer pass i >= 1 reads: W when (passes - 1 - i) is even
    const bool first_to_W = passes >= 2 && ((passes - 2) & 1) == 0;
    uint32_t *k0out = passes == 1 ? (uint32_t *)nullptr : (first_to_W ? kW : kX);
    int32_t *v0out = passes == 1 ? bins->ids : (first_to_W ? vW : vX);
    uint64_t *k64 = passes == 1 ? bins->keys : (uint64_t *)nullptr;
    if (current_tuning().generate_entries) {
        int32_t *chunk_rank = (int32_t *)(ws + L.chunk_rank);
        hipLaunchKernelGGL(chunk_rank_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, st, rank_ids, offsets,
                           s->tiles_touched, n_splats, K, cap, chunk_rank);
        hipLaunchKernelGGL(onesweep_emit_kernel, dim3((unsigned)L.tile_nb), dim3(kSortBlock), 0, st, rank_ids,
                           offsets, (const int32_t *)chunk_rank, s->tiles_touched, (const int4 *)s->rect, cams,
                           (int)n_cams, n_splats, K, cap, ghist_tile, stat_tile, tickets + kDepthPasses, k0out,
                           v0out, k64, s->depth, err);
    } else {
        // the emitted entries go to the pair the first pass does not write
        const bool emit_to_X = passes >= 2 && first_to_W;
        uint32_t *ek = emit_to_X ? kX : kW;
        int32_t *ev = emit_to_X ? vX : vW;
        hipLaunchKernelGGL(emit_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, st, rank_ids, offsets,
                           s->tiles_touched, (const int4 *)s->rect, cams, (int)n_cams, n_splats, K, cap, ek, ev);
        hipLaunchKernelGGL(onesweep_kernel, dim3((unsigned)L.tile_nb), dim3(kSortBlock), 0, st, ek, ev, K, cap, 0,
                           ghist_tile, stat_tile, tickets + kDepthPasses, k0out, v0out, k64, s->depth, n_splats, 1,
                           err);
    }
    uint32_t *kin = first_to_W ? kW : kX;
    int32_t *vin = first_to_W ? vW : vX;
    for (int pass = 1; pass < passes; ++pass) {
        const bool last = pass == passes - 1;
        uint32_t *kout = kin == kW ? kX : kW;
        int32_t *vout = vin == vW ? vX : vW;
        hipLaunchKernelGGL(onesweep_kernel, dim3((unsigned)L.tile_nb), dim3(kSortBlock), 0, st, kin, vin, K, cap,
                           pass * kRadixBits, ghist_tile + pass * kRadix,
                           stat_tile + (int64_t)pass * L.tile_nb * kRadix, tickets + kDepthPasses + pass,
                           last ? (uint32_t *)nullptr : kout, last ? bins->ids : vout,
                           last ? bins->keys : (uint64_t *)nullptr, s->depth, n_splats, 1, err);
        kin = kout;
        vin = vout;
    }
    rc = check_launch("tile sort");
    if (rc != GS_OK) return rc;
    hipLaunchKernelGGL(ranges_kernel, dim3(grid_for(cap, 256)), dim3(256), 0, st, bins->keys, K, cap, bins->n_tiles,
                       bins->ranges);

    // 5. the work list; the sort's error word joins the overflow flag
    hipLaunchKernelGGL(err_fold_kernel, dim3(1), dim3(64), 0, st, bins->counters, (const int64_t *)err);
    return build_schedule(bins, st);
}
