// gs_bin_and_sort: tile binning and per-tile depth order (Sec. 2.2).
//
// The result is the list of (tile, depth, splat) entries sorted by the 64-bit key
// (global tile << 32) | float32 depth bits, equal keys in splat order -- the order a single
// stable LSD radix sort of those 64-bit keys produces. It is computed as two stable
// LDS-histogram radix sorts whose traffic does not grow with the 32 depth bits per entry:
//
//   1. depth sort of the V splats that touch a tile: one pass compacts them in slot order
//      (32-bit keys = float bits of t_z, values = splat slot) and counts the digits of
//      every pass; then four 8-bit passes over V keys. Ties keep slot order.
//   2. exclusive scan of tiles_touched in depth-rank order -> per-rank emit offsets and
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
// Every sort pass and the range scan are single-pass launches with decoupled look-back:
// each block publishes its chunk's count(s), sums its predecessors' published counts for
// its global offsets (waiting, with a spin limit, on any predecessor that has not published
// yet) and writes its part. A sort pass ranks its chunk, stages it in LDS in digit order and
// writes it out in runs; the digit counts of all its passes come from one earlier read of
// the keys. The compaction and the emit-offset scan are three launches each in which no
// block waits on another (counts, a one-block scan, writes).
// Block ranking groups equal digits of a row of 64 keys with wave ballots; one leader lane
// per group adds the group's size to an LDS counter per (wave, digit), so atomics on a
// popular digit do not contend across lanes. Every kernel is sized from host-known
// capacities and reads its element count from device memory, and the look-back state is
// cleared by a kernel at the start of each call, so the whole sequence replays unchanged
// inside a captured HIP graph.
#include <mutex>

#include "common.h"

namespace gsx {

// ------------------------------------------------------------------------------ scan

constexpr int kScanBlock = 256;

// The value of another lane through a DPP move (0 where the control names no source lane or
// the row is masked off). Controls used: row_shr:n (0x110 + n, within rows of 16 lanes),
// row_bcast:15 (0x142, lane 15 of each row to the next row) and row_bcast:31 (0x143, lane
// 31 to rows 2 and 3).
template <int Ctrl, int RowMask, typename T>
__device__ inline T dpp_lane(T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, false);
    } else {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, Ctrl, RowMask, 0xf, false);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), Ctrl, RowMask, 0xf, false);
        return (T)(((uint64_t)hi << 32) | lo);
    }
}

// Inclusive prefix sum over the 64 lanes of a wave: scans within rows of 16 lanes (shifts by
// 1, 2, 4, 8), then each row's total carried into the rows above it (two row broadcasts).
template <typename T>
__device__ inline T wave_scan_incl(T v)
{
    v += dpp_lane<0x111, 0xf>(v);
    v += dpp_lane<0x112, 0xf>(v);
    v += dpp_lane<0x114, 0xf>(v);
    v += dpp_lane<0x118, 0xf>(v);
    v += dpp_lane<0x142, 0xa>(v);
    v += dpp_lane<0x143, 0xc>(v);
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive prefix and the
// block total through *total.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *total)
{
    __shared__ T wave_tot[kScanBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const T incl = wave_scan_incl(v);
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

// ------------------------------------------------------------------------ radix sort

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kSortItems = 16;                       // keys per lane
constexpr int kSortChunk = kSortBlock * kSortItems;  // keys per block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kMaxTilePassesDev = 4;   // tile ids are int32: at most four 8-bit passes
constexpr int kDepthPasses = 4;        // depth keys are 32-bit float bits
static_assert(kSortBlock == kRadix, "one thread per digit in the single-pass sort");

// A splat whose box has more than big_tiles tiles (launch tuning; 0: none) is listed by the
// per-tile merge instead of the tile sort.
__device__ inline bool is_big(int tiles, int big_tiles) { return big_tiles > 0 && tiles > big_tiles; }

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
// Per bit: the ballot of the lanes with the bit set, xor this lane's bit spread over 64
// bits, marks the lanes that differ from this one in that bit.
__device__ inline uint64_t match_digit(unsigned digit, uint64_t valid)
{
    uint64_t differ = 0;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const int bit = ((int)(digit << (31 - b))) >> 31;   // 0 or -1
        differ |= __ballot(bit != 0) ^ (uint64_t)(int64_t)bit;
    }
    return valid & ~differ;
}

// Ranks the keys of this block's chunk within their wave: rank[r] is the number of the
// wave's keys with the same digit before row r's key (earlier rows, then lower lanes of the
// same row); row r of wave w holds the chunk's keys w * M + 64 r + lane (M = kSortChunk /
// kSortWaves), valid below kvalid - chunk_base. Per row, the leader lane of each digit group
// adds the group's size to cnt[wave][digit] with an LDS atomic that returns the count
// before it, and the group takes that value from its leader. The atomics of a wave execute
// in issue order (the wave barrier keeps the compiler from reordering rows); all rows issue
// their atomics before any row reads a result back, so the rows do not wait on each other.
// Afterwards cnt[wave][digit] holds the wave's digit counts.
__device__ inline void rank_digits(const uint32_t (&key)[kSortItems], int64_t chunk_base, int64_t kvalid, int shift,
                                   unsigned (*cnt)[kRadix], unsigned (&rank)[kSortItems])
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint64_t lt = lanemask_lt();
    unsigned group = (unsigned)lane;   // previous row: leader lane | (peers below this lane) << 8
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const bool ok = chunk_base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane < kvalid;
        const uint64_t valid = __ballot(ok);
        rank[r] = 0;
        unsigned g = (unsigned)lane;
        if (valid != 0) {   // uniform
            const unsigned d = (key[r] >> shift) & (kRadix - 1);
            const uint64_t peers = match_digit(d, valid);
            if (ok && (peers & lt) == 0)
                rank[r] = __hip_atomic_fetch_add(&cnt[wave][d], (unsigned)__popcll(peers), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_wave_barrier();
            if (ok) g = (unsigned)__builtin_ctzll(peers) | ((unsigned)__popcll(peers & lt) << 8);
        }
        // the previous row's result is taken from its leader once this row's atomic is issued
        if (r > 0) rank[r - 1] = (unsigned)__shfl((int)rank[r - 1], (int)(group & 0xff), kWave) + (group >> 8);
        group = g;
    }
    rank[kSortItems - 1] = (unsigned)__shfl((int)rank[kSortItems - 1], (int)(group & 0xff), kWave) + (group >> 8);
}

// Status word of one (block, digit) in a single-pass sort, or of one block in a
// single-pass scan: 0 = not yet published, kStatAgg | the block's own count, kStatInc |
// inclusive prefix (for a sort: global position one past the block's last key with that
// digit).
constexpr uint64_t kStatAgg = 1ull << 62;
constexpr uint64_t kStatInc = 2ull << 62;
constexpr uint64_t kStatValue = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 20;   // bounded wait: a predecessor that never publishes ends the wait

// Polls a look-back wait makes before it gives up (gs_set_sort_wait_limit; kSpinLimit by
// default). A negative value makes every look-back give up at once, which lets a caller
// drive the give-up path (flag 2, no list) with every kernel ending normally.
__constant__ int g_wait_limit = kSpinLimit;

// True when look-backs are to give up at once (a negative wait limit); sets the error word.
__device__ inline bool forced_give_up(int64_t *err_flag)
{
    if (g_wait_limit >= 0) return false;
    __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Chunks of a single-pass launch are dealt to a grid of blocks that are all resident at
// once: block g takes chunks g, g + G, g + 2G, ... (G = gridDim.x) in turn. A chunk only
// waits on lower chunks, which are held by running blocks, so every wait ends without a
// global ticket counter (one atomic per chunk on a single address, which serialises the
// launch on this device). The grid fills the GPU when the chunks outnumber it, so nothing
// may run beside such a launch: a concurrent kernel would hold back some of its blocks while
// the others wait on their chunks. Called at the top of each turn: returns true when an earlier
// step of the sequence gave up (the error word is set); the block then stops.
__device__ inline bool chunk_stop(const int64_t *err_flag, int *sh_flag)
{
    __syncthreads();   // the previous turn's use of LDS has ended
    if (threadIdx.x == 0) *sh_flag = __hip_atomic_load(err_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    __syncthreads();
    return *sh_flag != 0;
}

// Gives up a look-back wait after g_wait_limit polls, or early once another block has given
// up (checked every 64 polls). Returns true when the wait is to end.
__device__ inline bool spin_exhausted(int &spins, int64_t *err_flag)
{
    ++spins;
    if (spins > g_wait_limit ||
        ((spins & 63) == 0 && __hip_atomic_load(err_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    __builtin_amdgcn_s_sleep(1);
    return false;
}

// Exclusive prefix of chunk b > 0 of a single-pass scan, from the status words of chunks
// 0 .. b - 1. Executed by the whole block (kSortBlock threads): thread t reads chunk j - t,
// so each step looks kSortBlock chunks back; the prefix is the sum of the values up to the
// nearest inclusive one. Every thread returns the prefix, or -1 when the wait gave up.
__device__ inline int64_t chained_prefix(const uint64_t *status, int b, int64_t *err_flag)
{
    __shared__ uint64_t s_inc[kSortWaves], s_nr[kSortWaves];
    __shared__ int64_t s_sum[kSortWaves];
    __shared__ int s_stop;
    if (forced_give_up(err_flag)) return -1;   // uniform: every thread reads the same constant
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int64_t acc = 0;
    int j = b - 1;
    int spins = 0;
    while (true) {
        const int idx = j - (int)threadIdx.x;
        const uint64_t st =
            idx >= 0 ? __hip_atomic_load(status + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kStatInc;
        const uint64_t flag = st & ~kStatValue;
        const uint64_t inc = __ballot(flag == kStatInc), nr = __ballot(flag == 0);
        if (lane == 0) {
            s_inc[wave] = inc;
            s_nr[wave] = nr;
        }
        __syncthreads();
        int first = kSortBlock;   // position of the nearest inclusive chunk in this window
        bool blocked = false;     // a chunk up to it has not published yet
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            if (first < kSortBlock) break;
            const uint64_t iw = s_inc[w], low = iw & (~iw + 1);
            if (s_nr[w] & (iw ? (low | (low - 1)) : ~0ull)) blocked = true;
            if (iw) first = w * kWave + __builtin_ctzll(iw);
        }
        if (blocked) {   // uniform: every thread read the same words
            if (threadIdx.x == 0) s_stop = spin_exhausted(spins, err_flag) ? 1 : 0;
            __syncthreads();
            if (s_stop) return -1;
            continue;
        }
        int64_t v = (int)threadIdx.x <= first ? (int64_t)(st & kStatValue) : 0;
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
        if (lane == 0) s_sum[wave] = v;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) acc += s_sum[w];
        __syncthreads();   // the window's shared words are rewritten by the next step
        if (first < kSortBlock) return acc;
        j -= kSortBlock;
    }
}

// Exclusive prefix, over chunks 0 .. b - 1 (b > 0), of digit d's counts in a single-pass
// sort, from their status words. The first step reads the nearest predecessor only (when
// chunks finish in order it is already inclusive, and the walk costs one load); later
// steps read kLookWindow chunks at once (independent loads whose latencies overlap) and sum
// down to the nearest inclusive word. When a chunk has not published yet, the sum keeps
// what lies above it and the next step starts there. Returns -1 when the wait gave up.
constexpr int kLookWindow = 8;

__device__ inline int64_t digit_lookback(const uint64_t *status, int b, int d, int64_t *err_flag)
{
    if (forced_give_up(err_flag)) return -1;
    int64_t acc = 0;
    int j = b - 1;   // highest chunk not yet summed
    int window = 1;
    int spins = 0;
    while (true) {
        uint64_t st[kLookWindow];
#pragma unroll
        for (int i = 0; i < kLookWindow; ++i) {
            // chunk 0 always publishes an inclusive word, so the walk never passes below it;
            // a zero word past the window ends the step like an unpublished chunk
            st[i] = 0;
            if (i < window)
                st[i] = j - i >= 0 ? __hip_atomic_load(status + (int64_t)(j - i) * kRadix + d, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT)
                                   : kStatInc;
        }
        int64_t sum = 0;
        int taken = 0;         // leading chunks of the window summed
        bool done = false, open = true;
#pragma unroll
        for (int i = 0; i < kLookWindow; ++i) {
            const uint64_t flag = st[i] & ~kStatValue;
            if (open && flag == 0) open = false;
            if (open) {
                sum += (int64_t)(st[i] & kStatValue);
                ++taken;
                if (flag == kStatInc) {
                    done = true;
                    open = false;
                }
            }
        }
        acc += sum;
        if (done) return acc;
        j -= taken;
        if (taken < window && spin_exhausted(spins, err_flag)) return -1;
        window = kLookWindow;
    }
}

// LDS of one single-pass sort block.
struct SweepShared {
    unsigned cnt[kSortWaves][kRadix];   // per-(wave, digit) counts, then staging cursors
    int64_t gdelta[kRadix];             // global position minus staging index, per digit
    uint32_t skey[kSortChunk];          // staged keys (digit order); first holds rank offsets
    int32_t sval[kSortChunk];
    int chunk, gave_up;
};

// Start of a turn: clears the counters; true when the block is to stop (see chunk_stop).
__device__ inline bool sweep_begin(SweepShared &sh, const int64_t *err_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) sh.gave_up = 0;
    for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortBlock) (&sh.cnt[0][0])[d] = 0;
    return chunk_stop(err_flag, &sh.chunk);
}

// Global position of the first key with digit d (thread d's value), from the pass's digit
// histogram; the same for every chunk of a launch.
__device__ inline int64_t digit_start(const unsigned *__restrict__ ghist)
{
    int64_t total;
    return block_exclusive_scan<int64_t>((int64_t)ghist[threadIdx.x], &total);
}

// Writes out staged keys q0 * kSortBlock + threadIdx.x, stepping by kSortBlock, kOutGroup of
// them: consecutive threads take consecutive staged keys, so each digit's run of the chunk
// is written by consecutive lanes to consecutive addresses, and all reads of the group
// (LDS, then the gathers) are issued before its writes.
constexpr int kOutGroup = 8;

__device__ inline void sweep_write(SweepShared &sh, int q0, int n_here, int64_t kvalid, int shift,
                                   uint32_t *__restrict__ keys_out, int32_t *__restrict__ vals_out,
                                   uint64_t *__restrict__ keys64_out, const float *__restrict__ depth,
                                   const int32_t *__restrict__ gather_src, int32_t *__restrict__ gather_dst,
                                   int64_t n_splats)
{
    uint32_t k_[kOutGroup];
    int32_t v_[kOutGroup];
    int64_t g_[kOutGroup];
#pragma unroll
    for (int q = 0; q < kOutGroup; ++q) {
        const int i = (int)threadIdx.x + (q0 + q) * kSortBlock;
        const bool ok = i < n_here;
        k_[q] = ok ? sh.skey[i] : 0u;
        v_[q] = ok ? sh.sval[i] : 0;
        g_[q] = ok ? sh.gdelta[(k_[q] >> shift) & (kRadix - 1)] + i : -1;
        if (g_[q] >= kvalid) g_[q] = -1;   // unreachable when the counts are consistent
    }
    if (keys64_out) {
        // v is a splat slot by construction; the test keeps a broken invariant from turning
        // into a wild read
        uint32_t dbits[kOutGroup];
#pragma unroll
        for (int q = 0; q < kOutGroup; ++q)
            dbits[q] = g_[q] >= 0 && (uint64_t)(uint32_t)v_[q] < (uint64_t)n_splats ? __float_as_uint(depth[v_[q]]) : 0u;
#pragma unroll
        for (int q = 0; q < kOutGroup; ++q) {
            if (g_[q] < 0) continue;
            vals_out[g_[q]] = v_[q];
            keys64_out[g_[q]] = ((uint64_t)k_[q] << 32) | (uint64_t)dbits[q];
        }
    } else {
        int32_t gs[kOutGroup];
        if (gather_dst) {
#pragma unroll
            for (int q = 0; q < kOutGroup; ++q)
                gs[q] = g_[q] >= 0 && (uint64_t)(uint32_t)v_[q] < (uint64_t)n_splats ? gather_src[v_[q]] : 0;
        }
#pragma unroll
        for (int q = 0; q < kOutGroup; ++q) {
            if (g_[q] < 0) continue;
            vals_out[g_[q]] = v_[q];
            if (keys_out) keys_out[g_[q]] = k_[q];
            if (gather_dst) gather_dst[g_[q]] = gs[q];
        }
    }
}

// One stable LSD pass over chunk b, keys already in registers in the wave-strided layout
// (lane l of wave w holds, in row r, key base + w * kSortChunk / kSortWaves + 64 r + l).
// The block ranks its chunk (rank_digits), publishes its digit counts, looks back over its
// predecessors' published counts for its global offsets, stages the chunk in LDS in digit
// order and writes it out in runs. dstart is digit_start of the pass. With keys64_out set
// (the last tile pass) it writes ids and the 64-bit keys (tile << 32 | depth bits of the
// value) instead of 32-bit keys; with gather_dst set it also writes gather_src[value] there
// in output order (keys_out may then be null).
__device__ inline void sweep_body(SweepShared &sh, const uint32_t (&key)[kSortItems],
                                  const int32_t (&val)[kSortItems], int b, int64_t base, int64_t kvalid, int shift,
                                  int64_t dstart, uint64_t *__restrict__ status,
                                  uint32_t *__restrict__ keys_out, int32_t *__restrict__ vals_out,
                                  uint64_t *__restrict__ keys64_out, const float *__restrict__ depth,
                                  const int32_t *__restrict__ gather_src, int32_t *__restrict__ gather_dst,
                                  int64_t n_splats, int64_t *__restrict__ err_flag)
{
    const int n_here = (int)min((int64_t)kSortChunk, kvalid - base);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    unsigned rank[kSortItems];
    rank_digits(key, base, kvalid, shift, sh.cnt, rank);
    __syncthreads();

    // thread d owns digit d
    const int d = threadIdx.x;
    unsigned tot = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) tot += sh.cnt[w][d];
    uint64_t *my = status + (int64_t)b * kRadix + d;
    int64_t excl = dstart;
    if (b == 0) {
        __hip_atomic_store(my, kStatInc | (uint64_t)(dstart + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(my, kStatAgg | (uint64_t)tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t acc = digit_lookback(status, b, d, err_flag);
        if (acc < 0) sh.gave_up = 1;   // the word below stays well formed; nothing is written
        excl = acc < 0 ? 0 : acc;
        __hip_atomic_store(my, kStatInc | (uint64_t)(excl + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned ltot;
    const unsigned ls = block_exclusive_scan<unsigned>(tot, &ltot);   // staging start of digit d
    sh.gdelta[d] = excl - (int64_t)ls;
    // per-(wave, digit) staging bases
    unsigned run = ls;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
        const unsigned c = sh.cnt[w][d];
        sh.cnt[w][d] = run;
        run += c;
    }
    __syncthreads();
    if (sh.gave_up) return;   // offsets unknown: write nothing (the error word is set)

    // stage the chunk in digit order (stable: waves in order, then rows, then lanes)
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
        if (idx < kvalid) {
            const unsigned pos = sh.cnt[wave][(key[r] >> shift) & (kRadix - 1)] + rank[r];
            sh.skey[pos] = key[r];
            sh.sval[pos] = val[r];
        }
    }
    __syncthreads();

    // write out (sweep_write)
#pragma unroll 1
    for (int q0 = 0; q0 < kSortItems; q0 += kOutGroup)
        sweep_write(sh, q0, n_here, kvalid, shift, keys_out, vals_out, keys64_out, depth, gather_src, gather_dst,
                    n_splats);
}

// One stable LSD pass with decoupled look-back (chained scan over chunks), in one launch of
// resident blocks (chunk_stop).
__global__ __launch_bounds__(kSortBlock) void onesweep_kernel(const uint32_t *__restrict__ keys_in,
                                                              const int32_t *__restrict__ vals_in,
                                                              const int64_t *__restrict__ count, int64_t cap,
                                                              int shift, const unsigned *__restrict__ ghist,
                                                              uint64_t *__restrict__ status,
                                                              uint32_t *__restrict__ keys_out,
                                                              int32_t *__restrict__ vals_out,
                                                              uint64_t *__restrict__ keys64_out,
                                                              const float *__restrict__ depth,
                                                              const int32_t *__restrict__ gather_src,
                                                              int32_t *__restrict__ gather_dst,
                                                              int64_t n_splats, int all_or_none,
                                                              int64_t *__restrict__ err_flag)
{
    __shared__ SweepShared sh;
    const int64_t kvalid = all_or_none ? tile_sort_count(count, cap) : sort_count(count, cap);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t dstart = digit_start(ghist);
    for (int64_t b = blockIdx.x; b * kSortChunk < kvalid; b += gridDim.x) {
        // the keys are loaded first, so their latency overlaps the turn's barriers
        const int64_t base = b * kSortChunk;
        uint32_t key[kSortItems];
        int32_t val[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t idx = base + (int64_t)wave * (kSortChunk / kSortWaves) + r * kWave + lane;
            const bool ok = idx < kvalid;
            key[r] = ok ? keys_in[idx] : 0u;
            val[r] = ok ? vals_in[idx] : 0;
        }
        if (sweep_begin(sh, err_flag)) break;
        sweep_body(sh, key, val, (int)b, base, kvalid, shift, dstart, status, keys_out, vals_out, keys64_out, depth,
                   gather_src, gather_dst, n_splats, err_flag);
        if (sh.gave_up) break;   // uniform: set before a barrier inside sweep_body
    }
}

// The first tile pass, over entries it generates itself: list entry k belongs to the splat
// of depth rank r with offsets[r] <= k < offsets[r] + tiles, as its (k - offsets[r])-th box
// tile in row-major order; its key is the global tile id and its value the splat slot. The
// block reads the rank offsets of its chunk into LDS, each thread generates 16 consecutive
// entries (one search for the first, then walking the box), and the chunk is regrouped
// into the strided layout of the ranking.
__global__ __launch_bounds__(kSortBlock) void onesweep_emit_kernel(
    const int32_t *__restrict__ rank_ids, const int64_t *__restrict__ offsets, const int32_t *__restrict__ chunk_rank,
    const int32_t *__restrict__ rank_tiles, const int4 *__restrict__ rect, const gs_camera *__restrict__ cams,
    int n_cams, int64_t n_splats, const int64_t *__restrict__ vcount, const int64_t *__restrict__ count, int64_t cap,
    const unsigned *__restrict__ ghist, uint64_t *__restrict__ status, uint32_t *__restrict__ keys_out,
    int32_t *__restrict__ vals_out, uint64_t *__restrict__ keys64_out, const float *__restrict__ depth,
    int64_t *__restrict__ err_flag)
{
    __shared__ SweepShared sh;
    __shared__ int n_ranks;
    const int64_t kvalid = tile_sort_count(count, cap);
    const int64_t n_chunks = (kvalid + kSortChunk - 1) / kSortChunk;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t dstart = digit_start(ghist);
    for (int64_t b = blockIdx.x; b < n_chunks; b += gridDim.x) {
        if (sweep_begin(sh, err_flag)) break;
        const int64_t base = b * kSortChunk;
        const int n_here = (int)min((int64_t)kSortChunk, kvalid - base);
        const int r0 = chunk_rank[b];
        if (threadIdx.x == 0) {
            const int64_t V = *vcount;
            const int64_t r_end = b + 1 < n_chunks ? (int64_t)chunk_rank[b + 1] : V - 1;
            n_ranks = (int)min((int64_t)kSortChunk, r_end - r0 + 1);
            // a rank outside [0, V) would mean inconsistent counts: report, write nothing
            if (r0 < 0 || r0 >= V || r_end < r0 || r_end >= V || V > n_splats) {
                n_ranks = 0;
                __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
        const int nr = n_ranks;
        if (nr == 0) break;   // uniform; blocks waiting on this chunk see the error word and stop
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
            int ntile = rank_tiles[r0 + ri];
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
                    ntile = rank_tiles[r0 + ri];
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
        sweep_body(sh, key, val, (int)b, base, kvalid, 0, dstart, status, keys_out, vals_out, keys64_out, depth,
                   (const int32_t *)nullptr, (int32_t *)nullptr, n_splats, err_flag);
        if (sh.gave_up) break;
    }
}

// ------------------------------------------------------------------- depth order, emit

// Depth keys of the splats that touch at least one tile, compacted in slot order: key =
// float bits of t_z (positive, so bit order is value order), value = slot. Three launches
// in which no block waits on another: per-chunk counts of the visible slots (chunks of
// kSortChunk slots), their exclusive scan (one block, which also stores V), then every
// chunk writes its kept keys at its offset; depth_hist_kernel then counts the digits of
// every depth pass over them.

// Visible slots among chunk c's kSortChunk slots (wave w, row r, lane l holds slot
// c * kSortChunk + w * M + 64 r + l, M = kSortChunk / kSortWaves).
__device__ inline unsigned chunk_visible(const int32_t *__restrict__ tiles, int64_t n, int64_t c,
                                         uint64_t (&vis)[kSortItems])
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t wbase = c * kSortChunk + (int64_t)wave * (kSortChunk / kSortWaves);
    unsigned mine = 0;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = wbase + r * kWave + lane;
        vis[r] = __ballot(idx < n && tiles[idx] > 0);
        mine += (unsigned)__popcll(vis[r]);
    }
    return mine;   // this wave's count
}

__global__ __launch_bounds__(kSortBlock) void visible_count_kernel(const int32_t *__restrict__ tiles, int64_t n,
                                                                   int32_t *__restrict__ chunk_cnt)
{
    __shared__ unsigned wave_tot[kSortWaves];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t n_chunks = (n + kSortChunk - 1) / kSortChunk;
    for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        uint64_t vis[kSortItems];
        const unsigned mine = chunk_visible(tiles, n, c, vis);
        __syncthreads();
        if (lane == 0) wave_tot[wave] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned t = 0;
#pragma unroll
            for (int w = 0; w < kSortWaves; ++w) t += wave_tot[w];
            chunk_cnt[c] = (int32_t)t;
        }
    }
}

// One block: exclusive scan in place of the per-chunk values of n_items items (chunks of
// kSortChunk; n_items from *n_dev when given), a contiguous run of chunks per thread. The
// total goes to *total and, when flag is given, (total > cap) to *flag.
template <typename T>
__global__ __launch_bounds__(kScanBlock) void chunk_scan_kernel(T *__restrict__ val, int64_t n_items,
                                                                const int64_t *__restrict__ n_dev,
                                                                int64_t *__restrict__ total,
                                                                int64_t *__restrict__ flag, int64_t cap)
{
    const int64_t items = n_dev ? *n_dev : n_items;
    const int64_t n_chunks = (items + kSortChunk - 1) / kSortChunk;
    const int64_t per = (n_chunks + kScanBlock - 1) / kScanBlock;
    const int64_t s0 = min(n_chunks, (int64_t)threadIdx.x * per), s1 = min(n_chunks, s0 + per);
    int64_t sum = 0;
    for (int64_t i = s0; i < s1; ++i) sum += val[i];
    int64_t tot;
    int64_t run = block_exclusive_scan<int64_t>(sum, &tot);
    for (int64_t i = s0; i < s1; ++i) {
        const T v = val[i];
        val[i] = (T)run;
        run += v;
    }
    if (threadIdx.x == 0) {
        *total = tot;
        if (flag) *flag = tot > cap ? 1 : 0;
    }
}

__global__ __launch_bounds__(kSortBlock) void visible_write_kernel(
    const int32_t *__restrict__ tiles, const float *__restrict__ depth, int64_t n,
    const int32_t *__restrict__ chunk_off, uint32_t *__restrict__ dkey, int32_t *__restrict__ dval)
{
    __shared__ unsigned wave_tot[kSortWaves];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t n_chunks = (n + kSortChunk - 1) / kSortChunk;
    for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        uint64_t vis[kSortItems];
        const unsigned mine = chunk_visible(tiles, n, c, vis);
        __syncthreads();   // the previous chunk's use of wave_tot has ended
        if (lane == 0) wave_tot[wave] = mine;
        __syncthreads();
        unsigned before = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w)
            if (w < wave) before += wave_tot[w];
        const int64_t prefix = chunk_off[c];
        const int64_t wbase = c * kSortChunk + (int64_t)wave * (kSortChunk / kSortWaves);
        unsigned local = before;   // block-local position of the wave's next kept key
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            if ((vis[r] >> lane) & 1) {
                const int64_t idx = wbase + r * kWave + lane;
                const unsigned l = local + (unsigned)__popcll(vis[r] & lanemask_lt());
                dkey[prefix + l] = __float_as_uint(depth[idx]);
                dval[prefix + l] = (int32_t)idx;
            }
            local += (unsigned)__popcll(vis[r]);
        }
    }
}

// Digit counts of every depth pass over the V compacted keys: per-wave LDS histograms
// (LDS atomics contend only within a wave), added to ghist[pass][digit] once per block.
__global__ __launch_bounds__(kSortBlock) void depth_hist_kernel(const uint32_t *__restrict__ dkey,
                                                                const int64_t *__restrict__ vcount,
                                                                unsigned *__restrict__ ghist)
{
    __shared__ unsigned h[kSortWaves][kDepthPasses][kRadix];
    const int wave = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kSortWaves * kDepthPasses * kRadix; i += kSortBlock) (&h[0][0][0])[i] = 0;
    __syncthreads();
    const int64_t V = *vcount;
    constexpr int kU = 8;
    for (int64_t i0 = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; i0 < V;
         i0 += (int64_t)gridDim.x * kSortBlock * kU) {
        uint32_t k[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = i0 + (int64_t)u * gridDim.x * kSortBlock;
            k[u] = i < V ? dkey[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (i0 + (int64_t)u * gridDim.x * kSortBlock >= V) continue;
#pragma unroll
            for (int pass = 0; pass < kDepthPasses; ++pass)
                atomicAdd(&h[wave][pass][(k[u] >> (pass * kRadixBits)) & (kRadix - 1)], 1u);
        }
    }
    __syncthreads();
    const int d = threadIdx.x;   // kSortBlock == kRadix
#pragma unroll
    for (int pass = 0; pass < kDepthPasses; ++pass) {
        unsigned tot = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) tot += h[w][pass][d];
        if (tot) atomicAdd(&ghist[pass * kRadix + d], tot);
    }
}

// Emit offsets: exclusive scan of tiles_touched in depth-rank order over the V visible
// splats (rank_tiles, written in rank order by the last depth pass). Chunks of kSortChunk
// ranks, 16 consecutive ranks per thread: per-chunk sums, their scan (chunk_scan_kernel,
// which stores K and the overflow flag), then each chunk writes its offsets.
// Tile counts of ranks i0 .. i0 + 15 (0 past V, and 0 for splats listed by the merge).
__device__ inline void load_rank_tiles(const int32_t *__restrict__ rank_tiles, int64_t i0, int64_t V,
                                       int32_t (&t)[kSortItems], int big_tiles)
{
    if (i0 + kSortItems <= V) {
        const int4 *t4 = reinterpret_cast<const int4 *>(rank_tiles + i0);
#pragma unroll
        for (int q = 0; q < kSortItems / 4; ++q) {
            const int4 v = t4[q];
            t[4 * q] = v.x; t[4 * q + 1] = v.y; t[4 * q + 2] = v.z; t[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) t[k] = i0 + k < V ? rank_tiles[i0 + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k)
        if (is_big(t[k], big_tiles)) t[k] = 0;
}

__global__ __launch_bounds__(kSortBlock) void rank_sum_kernel(const int32_t *__restrict__ rank_tiles,
                                                              const int64_t *__restrict__ vcount,
                                                              int64_t *__restrict__ chunk_sum, int big_tiles)
{
    const int64_t V = *vcount;
    for (int64_t c = blockIdx.x; c * kSortChunk < V; c += gridDim.x) {
        int32_t t[kSortItems];
        load_rank_tiles(rank_tiles, c * kSortChunk + (int64_t)threadIdx.x * kSortItems, V, t, big_tiles);
        int64_t mine = 0;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) mine += t[k];
        int64_t tot;
        block_exclusive_scan<int64_t>(mine, &tot);
        if (threadIdx.x == 0) chunk_sum[c] = tot;
    }
}

__global__ __launch_bounds__(kSortBlock) void rank_offsets_kernel(const int32_t *__restrict__ rank_tiles,
                                                                  const int64_t *__restrict__ vcount,
                                                                  const int64_t *__restrict__ chunk_off,
                                                                  int64_t *__restrict__ offsets, int big_tiles)
{
    const int64_t V = *vcount;
    for (int64_t c = blockIdx.x; c * kSortChunk < V; c += gridDim.x) {
        const int64_t i0 = c * kSortChunk + (int64_t)threadIdx.x * kSortItems;
        int32_t t[kSortItems];
        load_rank_tiles(rank_tiles, i0, V, t, big_tiles);
        int64_t mine = 0;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) mine += t[k];
        int64_t tot;
        int64_t run = block_exclusive_scan<int64_t>(mine, &tot) + chunk_off[c];
        if (i0 + kSortItems <= V) {
            longlong2 *o2 = reinterpret_cast<longlong2 *>(offsets + i0);
#pragma unroll
            for (int q = 0; q < kSortItems / 2; ++q) {
                longlong2 v;
                v.x = run;
                run += t[2 * q];
                v.y = run;
                run += t[2 * q + 1];
                o2[q] = v;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) {
                if (i0 + k < V) offsets[i0 + k] = run;
                run += t[k];
            }
        }
    }
}

// ----------------------------------------------------------- tile-pass histograms, emit

// ------------------------------------------------------- per-tile list lengths, ranges

// Every listed splat adds one entry to each tile of its box, so the list length of a tile
// is a 2D box count: per camera, +1 at (y0, x0) and (y1 + 1, x1 + 1) and -1 at (y0, x1 + 1)
// and (y1 + 1, x0) of a difference array over its tile grid (corners past the grid
// dropped), then 2D prefix sums. Each splat costs four LDS atomics whatever the size of its
// box. The lengths give the digit histograms of the tile passes (before them) and every
// tile's range (after them).
constexpr int kCountLds = 8192;     // LDS cells: one band of rows of a tile grid (1920x1080: 8160)
constexpr int kCornerBlock = 1024;

// A block takes `span` consecutive entries of the compacted visible slots (ascending, so
// each camera's slots are contiguous), adds their corners to an LDS difference array for
// each camera it meets (a grid of more than kCountLds tiles in bands of rows), and adds
// the nonzero cells to the global array, indexed by global tile id.
__global__ __launch_bounds__(kCornerBlock) void tile_corner_kernel(const int32_t *__restrict__ vis_slots,
                                                                   const int64_t *__restrict__ vcount,
                                                                   const int4 *__restrict__ rect,
                                                                   const gs_camera *__restrict__ cams, int n_cams,
                                                                   int64_t n_splats, int64_t span, int big_tiles,
                                                                   int32_t *__restrict__ gdiff)
{
    __shared__ int diff[kCountLds];
    const int64_t V = *vcount;
    const int64_t s0 = (int64_t)blockIdx.x * span;
    if (s0 >= V) return;   // uniform
    const int64_t s1 = min(s0 + span, V);
    const int c_first = camera_of_splat(cams, n_cams, vis_slots[s0]);
    const int c_last = camera_of_splat(cams, n_cams, vis_slots[s1 - 1]);
    constexpr int kU = 4;   // slots per thread in flight
    for (int c = c_first; c <= c_last; ++c) {
        const int64_t p_lo = max(cams[c].proj_offset, (int64_t)0);
        const int64_t p_hi = min(p_lo + cams[c].gauss_count, n_splats);
        const int W = cams[c].tiles_x, H = cams[c].tiles_y, toff = cams[c].tile_offset;
        if (W < 1 || H < 1 || W > kCountLds) continue;   // uniform; tile_count_kernel reports it
        const int band = kCountLds / W;
        for (int yb = 0; yb < H; yb += band) {
            const int rows = min(band, H - yb);
            for (int i = threadIdx.x; i < rows * W; i += kCornerBlock) diff[i] = 0;
            __syncthreads();
            for (int64_t i0 = s0 + threadIdx.x; i0 < s1; i0 += kU * kCornerBlock) {
                int32_t sl[kU];
                int4 bx[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int64_t i = i0 + (int64_t)u * kCornerBlock;
                    sl[u] = i < s1 ? vis_slots[i] : -1;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    bx[u] = sl[u] >= p_lo && sl[u] < p_hi ? rect[sl[u]] : make_int4(0, 0, -1, -1);
                    // splats listed by the merge are not counted here (their tiles are added later)
                    if (bx[u].z >= 0 && is_big((bx[u].z - bx[u].x + 1) * (bx[u].w - bx[u].y + 1), big_tiles))
                        bx[u] = make_int4(0, 0, -1, -1);
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if (bx[u].z < 0) continue;   // not this camera's slot
                    const int x0 = min(max(bx[u].x, 0), W - 1), x1 = min(max(bx[u].z, 0), W - 1) + 1;
                    const int y0 = min(max(bx[u].y, 0), H - 1), y1 = min(max(bx[u].w, 0), H - 1) + 1;
                    if (y0 >= yb && y0 < yb + rows) {
                        atomicAdd(&diff[(y0 - yb) * W + x0], 1);
                        if (x1 < W) atomicAdd(&diff[(y0 - yb) * W + x1], -1);
                    }
                    if (y1 < H && y1 >= yb && y1 < yb + rows) {
                        atomicAdd(&diff[(y1 - yb) * W + x0], -1);
                        if (x1 < W) atomicAdd(&diff[(y1 - yb) * W + x1], 1);
                    }
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < rows * W; i += kCornerBlock)
                if (diff[i]) atomicAdd(&gdiff[toff + (int64_t)yb * W + i], diff[i]);
            __syncthreads();
        }
    }
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ inline int wave_inclusive_scan(int v) { return wave_scan_incl(v); }

constexpr int kCountBlock = 1024;

// One block per camera: 2D prefix sums of its difference array (bands of rows in LDS; a
// wave scans a row, then a column, 64 cells at a time) give the list length of every tile,
// written over the difference array; the digit histograms of the tile passes are added
// from the lengths.
__global__ __launch_bounds__(kCountBlock) void tile_count_kernel(const gs_camera *__restrict__ cams, int passes,
                                                                 int32_t *__restrict__ cnt,
                                                                 unsigned *__restrict__ ghist,
                                                                 int64_t *__restrict__ err_flag)
{
    __shared__ int cells[kCountLds];
    __shared__ int col_run[kCountLds];
    __shared__ unsigned h[kMaxTilePassesDev][kRadix];
    constexpr int kWaves = kCountBlock / kWave;
    const int c = blockIdx.x;
    const int W = cams[c].tiles_x, H = cams[c].tiles_y, toff = cams[c].tile_offset;
    if (W > kCountLds) {   // uniform: wider than 131072 pixels is not supported
        if (threadIdx.x == 0) __hip_atomic_store(err_flag, (int64_t)4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    if (W < 1 || H < 1) return;   // uniform: no tiles
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kMaxTilePassesDev * kRadix; i += kCountBlock) (&h[0][0])[i] = 0;
    for (int i = threadIdx.x; i < W; i += kCountBlock) col_run[i] = 0;
    const int band = kCountLds / W;
    for (int yb = 0; yb < H; yb += band) {
        const int rows = min(band, H - yb), n = rows * W;
        const int64_t t0 = toff + (int64_t)yb * W;
        for (int i = threadIdx.x; i < n; i += kCountBlock) cells[i] = cnt[t0 + i];
        __syncthreads();
        for (int r = wave; r < rows; r += kWaves) {
            int carry = 0;
            for (int x0 = 0; x0 < W; x0 += kWave) {
                const int x = x0 + lane;
                const int v = wave_inclusive_scan(x < W ? cells[r * W + x] : 0) + carry;
                if (x < W) cells[r * W + x] = v;
                carry = __shfl(v, kWave - 1, kWave);
            }
        }
        __syncthreads();
        for (int x = wave; x < W; x += kWaves) {
            int carry = col_run[x];
            for (int r0 = 0; r0 < rows; r0 += kWave) {
                const int r = r0 + lane;
                const int v = wave_inclusive_scan(r < rows ? cells[r * W + x] : 0) + carry;
                if (r < rows) cells[r * W + x] = v;
                carry = __shfl(v, kWave - 1, kWave);
            }
            if (lane == 0) col_run[x] = carry;
        }
        __syncthreads();
        // a wave holds 64 consecutive tiles: their low digits differ, while a higher digit is
        // mostly the same across the wave, so it is added once from the wave's sum
        for (int b = 0; b < n; b += kCountBlock) {
            const int i = b + (int)threadIdx.x;
            const bool ok = i < n;
            const int v = ok ? cells[i] : 0;
            const int64_t t = t0 + i;
            if (ok) cnt[t] = v;
            if (v) atomicAdd(&h[0][t & (kRadix - 1)], (unsigned)v);
            for (int pass = 1; pass < passes; ++pass) {
                const unsigned d = (unsigned)(t >> (pass * kRadixBits)) & (kRadix - 1);
                const unsigned d0 = __builtin_amdgcn_readfirstlane(d);
                if (__ballot(ok && d != d0) == 0) {   // uniform
                    const int sum = __shfl(wave_inclusive_scan(v), kWave - 1, kWave);
                    if (lane == 0 && sum) atomicAdd(&h[pass][d0], (unsigned)sum);
                } else if (v) {
                    atomicAdd(&h[pass][d], (unsigned)v);
                }
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < passes * kRadix; i += kCountBlock)
        if ((&h[0][0])[i]) atomicAdd(&ghist[i], (&h[0][0])[i]);
}

// Ranges: exclusive scan of the list lengths in global tile order (single pass, chunks of
// kSortChunk tiles, 16 consecutive tiles per thread), run only when the list was built (K
// within the capacity, no error). A range is written only when it ends within K, so the
// rasterizer never reads past the list; a range past K, or a total different from K,
// marks the lengths inconsistent with the list (error word). Empty tiles get (0, 0).
// With big_len (the merge of large splats) the scan also gives big_before[t], the entries
// of big splats in tiles before t: each tile's value is packed as length << 31 | big count
// (both sums stay below 2^31 when the list is built, so the fields never carry into each
// other and the packed prefix fits the 62-bit status value).
constexpr int kPackShift = 31;
constexpr int64_t kPackLow = (1ll << kPackShift) - 1;

__global__ __launch_bounds__(kSortBlock) void ranges_kernel(const int32_t *__restrict__ cnt, int32_t n_tiles,
                                                            const int64_t *__restrict__ K, int64_t cap,
                                                            uint64_t *__restrict__ status,
                                                            int32_t *__restrict__ ranges,
                                                            const int32_t *__restrict__ big_len,
                                                            int32_t *__restrict__ big_before,
                                                            int64_t *__restrict__ err_flag)
{
    __shared__ int64_t prefix;
    __shared__ int stop;
    const int64_t k_all = *K;
    if (k_all > cap) return;   // uniform: the list was not built
    for (int64_t b = blockIdx.x; b * kSortChunk < n_tiles; b += gridDim.x) {
    if (chunk_stop(err_flag, &stop)) break;
    const int64_t base = b * kSortChunk;
    const int64_t i0 = base + (int64_t)threadIdx.x * kSortItems;
    int32_t n[kSortItems], nb[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        n[k] = i0 + k < n_tiles ? cnt[i0 + k] : 0;
        nb[k] = big_len && i0 + k < n_tiles ? big_len[i0 + k] : 0;
    }
    int64_t mine = 0;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) mine += ((int64_t)n[k] << kPackShift) + nb[k];
    int64_t total;
    const int64_t ex_thread = block_exclusive_scan<int64_t>(mine, &total);
    if (threadIdx.x == 0)
        __hip_atomic_store(status + b, (b == 0 ? kStatInc : kStatAgg) | (uint64_t)total, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    const int64_t ex = b == 0 ? 0 : chained_prefix(status, (int)b, err_flag);
    if (threadIdx.x == 0) {
        if (b > 0 && ex >= 0)
            __hip_atomic_store(status + b, kStatInc | (uint64_t)(ex + total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        prefix = ex;
        if (ex >= 0 && base + kSortChunk >= n_tiles && ((ex + total) >> kPackShift) != k_all)
            __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (prefix < 0) break;
    int64_t run = prefix + ex_thread;
    bool past = false;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t s0 = run >> kPackShift, e = s0 + n[k];
        if (i0 + k < n_tiles) {
            if (n[k] > 0 && e <= k_all) {
                ranges[2 * (i0 + k)] = (int32_t)s0;
                ranges[2 * (i0 + k) + 1] = (int32_t)e;
            } else if (n[k] > 0) {
                past = true;
            }
            if (big_before) big_before[i0 + k] = (int32_t)(run & kPackLow);
        }
        run += ((int64_t)n[k] << kPackShift) + nb[k];
    }
    if (past) __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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
// With big_tiles > 0, splats with more tiles than that are left out (the merge lists them)
// and the value of an entry is the splat's depth rank instead of its slot.
__global__ __launch_bounds__(256) void emit_kernel(const int32_t *__restrict__ rank_ids,
                                                   const int64_t *__restrict__ offsets,
                                                   const int32_t *__restrict__ rank_tiles, const int4 *__restrict__ rect,
                                                   const gs_camera *__restrict__ cams, int n_cams, int64_t n_splats,
                                                   const int64_t *__restrict__ vcount,
                                                   const int64_t *__restrict__ K, int64_t cap,
                                                   uint32_t *__restrict__ tkey, int32_t *__restrict__ tval,
                                                   int big_tiles, const int64_t *__restrict__ err_flag)
{
    if (*K > cap || *err_flag) return;   // uniform
    const int64_t V = *vcount;
    const int lane = threadIdx.x & (kWave - 1);
    // a grid of a few blocks per CU walks the V ranks (the grid is sized for the slots, of
    // which V may be a small part)
    for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x; r0 < V; r0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = r0 + threadIdx.x;
    int32_t slot = 0, val = 0;
    int cnt = 0;
    int64_t k0 = 0;
    if (r < V) {
        slot = rank_ids[r];
        cnt = rank_tiles[r];
        k0 = offsets[r];
        if (is_big(cnt, big_tiles)) cnt = 0;
        val = big_tiles > 0 ? (int32_t)r : slot;
    }
    int toff = 0, tx_n = 1;
    int4 b = make_int4(0, 0, 0, 0);
    if (cnt > 0) {
        const int c = camera_of_splat(cams, n_cams, slot);
        toff = cams[c].tile_offset;
        tx_n = cams[c].tiles_x;
        b = rect[slot];
    }
    if (cnt > 0 && cnt <= kEmitLaneMax) emit_tiles(k0, 0, 1, cnt, b, toff, tx_n, val, tkey, tval);
    // large boxes: the whole wave writes them, one splat at a time
    uint64_t big = __ballot(cnt > kEmitLaneMax);
    while (big) {
        const int src = __builtin_ctzll(big);
        big &= big - 1;
        const int bcnt = __shfl(cnt, src, kWave);
        const int64_t bk0 = __shfl(k0, src, kWave);
        const int32_t bslot = __shfl(val, src, kWave);
        const int btoff = __shfl(toff, src, kWave), btx = __shfl(tx_n, src, kWave);
        const int4 bb = make_int4(__shfl(b.x, src, kWave), __shfl(b.y, src, kWave), __shfl(b.z, src, kWave),
                                  __shfl(b.w, src, kWave));
        emit_tiles(bk0, lane, kWave, bcnt, bb, btoff, btx, bslot, tkey, tval);
    }
    }
}

// ------------------------------------------------------ the merge of large splats
//
// A splat that covers many tiles (typically one close to a camera) adds an entry to each of
// them, and such entries can be most of the list. With big_tiles > 0 the splats with more
// tiles than that are not emitted. Within a camera, the big splats listed in a tile are,
// in depth-rank order, the camera's big splats whose box contains the tile, so each tile's
// list is the merge by depth rank of two sorted runs: its run of the tile-sorted small
// entries (whose values are ranks) and that filtered run of big splats. Ranks are distinct,
// so the merge gives exactly the order of the full sort. Steps:
//   big_count   per chunk of ranks: big splats per camera, and the sum of their tiles;
//   big_scan    camera-major offsets of the big splats; K = small + big entries, overflow;
//   big_scatter the big splats per camera in rank order (rank, slot, camera-local box);
//   big_len     per tile, the big splats whose box contains it (added to the tile lengths;
//               the ranges scan also gives big_before, the big entries of earlier tiles);
//   merge       per tile, the merge of its small run with its filtered big splats, written
//               as ids (and keys).
constexpr int kBigMaxCams = 64;   // cameras per call for which the merge is used
constexpr int kBigMinTiles = 16;  // smallest big_tiles: the big splat arrays hold K_cap / 17
// words of the call's big-splat state (after the per-camera starts)
constexpr int kBigKSmall = 0;     // entries of small splats (written by the offset scan)
constexpr int kBigKBig = 1;       // entries of big splats (summed by big_count)
constexpr int kBigEffSmall = 2;   // entries the tile sort takes: K_small, or 0 when nothing is built
constexpr int kBigOk = 3;         // 1 when the list is built
constexpr int kBigCamStart = 8;   // [kBigMaxCams + 1] start of each camera's big splats
constexpr int kBigCamTotal = kBigCamStart + kBigMaxCams + 1;   // [kBigMaxCams] big splats per camera
constexpr int kBigWords = kBigCamTotal + kBigMaxCams;

// A big splat's camera-local tile box, x0 | y0 << 16 and x1 | y1 << 16 (tile coordinates
// below 2^16; a larger one makes the sort fail with flag 2 instead).
__device__ inline uint2 pack_box(const int4 &b)
{
    return make_uint2((uint32_t)b.x | ((uint32_t)b.y << 16), (uint32_t)b.z | ((uint32_t)b.w << 16));
}

// (all four compares evaluated: no branches between a load and its use)
__device__ inline bool box_holds(const uint2 &b, int tx, int ty)
{
    return ((int)(b.x & 0xffff) <= tx) & (tx <= (int)(b.y & 0xffff)) & ((int)(b.x >> 16) <= ty) &
           (ty <= (int)(b.y >> 16));
}

constexpr uint2 kEmptyBox = {1u, 0u};   // x0 = 1 > x1 = 0: holds no tile

// Per chunk c of kSortChunk ranks: the count of big splats of each camera (mat[cam * stride
// + c]; cameras' totals summed into words[kBigCamTotal + cam]) and the sum of their tiles
// (summed into words[kBigKBig]).
__global__ __launch_bounds__(kSortBlock) void big_count_kernel(const int32_t *__restrict__ rank_ids,
                                                               const int32_t *__restrict__ rank_tiles,
                                                               const int64_t *__restrict__ vcount,
                                                               const gs_camera *__restrict__ cams, int n_cams,
                                                               int big_tiles, int32_t *__restrict__ mat,
                                                               int64_t stride, int64_t *__restrict__ words,
                                                               const int64_t *__restrict__ err_flag)
{
    __shared__ int cnt[kBigMaxCams];
    if (*err_flag) return;   // uniform
    const int64_t V = *vcount;
    for (int64_t c = blockIdx.x; c * kSortChunk < V; c += gridDim.x) {
        __syncthreads();
        if (threadIdx.x < kBigMaxCams) cnt[threadIdx.x] = 0;
        __syncthreads();
        const int64_t i0 = c * kSortChunk + (int64_t)threadIdx.x * kSortItems;
        int32_t t[kSortItems];
        load_rank_tiles(rank_tiles, i0, V, t, 0);
        int64_t mine = 0;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            if (i0 + k < V && is_big(t[k], big_tiles)) {
                atomicAdd(&cnt[camera_of_splat(cams, n_cams, rank_ids[i0 + k])], 1);
                mine += t[k];
            }
        }
        int64_t tot;
        block_exclusive_scan<int64_t>(mine, &tot);
        if (threadIdx.x < n_cams) {
            const int v = cnt[threadIdx.x];
            mat[threadIdx.x * stride + c] = v;
            if (v) atomicAdd((unsigned long long *)(words + kBigCamTotal + threadIdx.x), (unsigned long long)v);
        }
        if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long *)(words + kBigKBig), (unsigned long long)tot);
    }
}

// One block per camera: its row of mat becomes the exclusive offsets of its big splats by
// chunk, starting at the totals of the cameras before it. Block 0 also stores every camera's
// start, sets K = K_small + K_big in counters[0] and the overflow flag in counters[1], and
// decides whether the list is built (kBigOk, and the tile sort's count).
__global__ __launch_bounds__(kScanBlock) void big_scan_kernel(int32_t *__restrict__ mat, int64_t stride,
                                                              const int64_t *__restrict__ vcount, int n_cams,
                                                              int64_t *__restrict__ words,
                                                              int64_t *__restrict__ counters, int64_t cap,
                                                              int64_t big_cap, int64_t *__restrict__ err_flag)
{
    const int cam = blockIdx.x;
    const int64_t V = *vcount;
    const int64_t n_chunks = (V + kSortChunk - 1) / kSortChunk;
    int64_t base = 0;
    for (int c = 0; c < cam; ++c) base += words[kBigCamTotal + c];
    int32_t *row = mat + cam * stride;
    for (int64_t b = 0; b < n_chunks; b += (int64_t)kScanBlock * kSortItems) {
        const int64_t i0 = b + (int64_t)threadIdx.x * kSortItems;
        int32_t v[kSortItems];
        int64_t mine = 0;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            v[k] = i0 + k < n_chunks ? row[i0 + k] : 0;
            mine += v[k];
        }
        int64_t tot;
        int64_t run = base + block_exclusive_scan<int64_t>(mine, &tot);
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            if (i0 + k < n_chunks) row[i0 + k] = (int32_t)run;
            run += v[k];
        }
        base += tot;
    }
    if (cam != 0 || threadIdx.x != 0) return;
    int64_t n_big = 0;
    for (int c = 0; c < n_cams; ++c) {
        words[kBigCamStart + c] = n_big;
        n_big += words[kBigCamTotal + c];
    }
    words[kBigCamStart + n_cams] = n_big;
    const int64_t k_small = words[kBigKSmall], total = k_small + words[kBigKBig];
    const bool over = total > cap;
    counters[0] = total;
    counters[1] = over ? 1 : 0;
    bool ok = !over && *err_flag == 0;
    if (ok && n_big > big_cap) {   // unreachable: each big splat adds more than kBigMinTiles entries
        __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
    }
    words[kBigOk] = ok ? 1 : 0;
    words[kBigEffSmall] = ok ? k_small : 0;
}

// Per chunk of ranks: the chunk's big splats in rank order (a block scan into LDS), then
// one wave gives each its place in its camera's run (lanes of one camera in lane order,
// each camera's cursor advanced by its group's leader): rank and camera-local box.
__global__ __launch_bounds__(kSortBlock) void big_scatter_kernel(const int32_t *__restrict__ rank_ids,
                                                                 const int32_t *__restrict__ rank_tiles,
                                                                 const int64_t *__restrict__ vcount,
                                                                 const gs_camera *__restrict__ cams, int n_cams,
                                                                 int big_tiles, const int4 *__restrict__ rect,
                                                                 const int32_t *__restrict__ mat, int64_t stride,
                                                                 const int64_t *__restrict__ words,
                                                                 int4 *__restrict__ big_rec,
                                                                 int64_t *__restrict__ err_flag)
{
    __shared__ int32_t lrank[kSortChunk];
    __shared__ int cursor[kBigMaxCams];
    if (!words[kBigOk] || *err_flag) return;   // uniform
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t V = *vcount, n_big = words[kBigCamStart + n_cams];
    for (int64_t c = blockIdx.x; c * kSortChunk < V; c += gridDim.x) {
        __syncthreads();   // the previous chunk's LDS reads have ended
        const int64_t i0 = c * kSortChunk + (int64_t)threadIdx.x * kSortItems;
        int32_t t[kSortItems];
        load_rank_tiles(rank_tiles, i0, V, t, 0);
        int mine = 0;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) mine += (i0 + k < V && is_big(t[k], big_tiles)) ? 1 : 0;
        int nb;
        int at = block_exclusive_scan<int>(mine, &nb);
#pragma unroll
        for (int k = 0; k < kSortItems; ++k)
            if (i0 + k < V && is_big(t[k], big_tiles)) lrank[at++] = (int32_t)(i0 + k);
        if (threadIdx.x < n_cams) cursor[threadIdx.x] = mat[threadIdx.x * stride + c];
        __syncthreads();
        if (wave != 0 || nb == 0) continue;   // wave-uniform; the next turn starts with a barrier
        for (int b = 0; b < nb; b += kWave) {
            const int i = b + lane;
            const bool ok = i < nb;
            const int32_t r = ok ? lrank[i] : 0;
            const int32_t slot = ok ? rank_ids[r] : 0;
            const int cam = ok ? camera_of_splat(cams, n_cams, slot) : 0;
            const uint64_t peers = match_digit((unsigned)cam, __ballot(ok));
            const int64_t pos = (int64_t)cursor[cam] + __popcll(peers & lanemask_lt());
            __builtin_amdgcn_wave_barrier();
            if (ok && pos >= 0 && pos < n_big) {   // always true when the counts agree
                const int4 b = rect[slot];
                if ((uint32_t)(b.x | b.y | b.z | b.w) > 0xffffu)
                    __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint2 pb = pack_box(b);
                big_rec[pos] = make_int4(r, slot, (int)pb.x, (int)pb.y);
            }
            if (ok && (peers & lanemask_lt()) == 0) cursor[cam] = (int)(pos + __popcll(peers));
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// One block per camera: its big splats' boxes (clipped to its grid) go into an LDS difference
// array over its tile grid, in bands of rows of at most kCountLds cells (a box enters a band
// at its first row inside it), and 2D prefix sums (a wave scans a row, then a column) give
// the number of boxes containing each tile: kept in big_len and added to the tile's list
// length. The same count as testing every tile against every box, in four LDS atomics per
// box and band.
__global__ __launch_bounds__(kCountBlock) void big_len_kernel(const gs_camera *__restrict__ cams, int n_cams,
                                                              const int64_t *__restrict__ words,
                                                              const int4 *__restrict__ big_rec,
                                                              int32_t *__restrict__ cnt, int32_t *__restrict__ big_len,
                                                              const int64_t *__restrict__ err_flag)
{
    __shared__ int cells[kCountLds];
    constexpr int kWaves = kCountBlock / kWave;
    if (!words[kBigOk] || *err_flag) return;   // uniform
    const int c = blockIdx.x;
    if (c >= n_cams) return;
    const int W = cams[c].tiles_x, H = cams[c].tiles_y, toff = cams[c].tile_offset;
    if (W < 1 || H < 1 || W > kCountLds) return;   // uniform; tile_count_kernel reports a grid too wide
    const int64_t b0 = words[kBigCamStart + c], b1 = words[kBigCamStart + c + 1];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int band = kCountLds / W;
    for (int yb = 0; yb < H; yb += band) {
        const int rows = min(band, H - yb), n = rows * W;
        for (int i = threadIdx.x; i < n; i += kCountBlock) cells[i] = 0;
        __syncthreads();
        for (int64_t k = b0 + threadIdx.x; k < b1; k += kCountBlock) {
            const int4 rec = big_rec[k];
            const uint2 b = make_uint2((uint32_t)rec.z, (uint32_t)rec.w);
            const int x0 = (int)(b.x & 0xffff), x1 = min((int)(b.y & 0xffff), W - 1);
            const int y0 = max((int)(b.x >> 16), yb), y1 = min((int)(b.y >> 16), H - 1);
            if (x0 > x1 || y0 > y1 || y0 >= yb + rows) continue;   // no tile of this band
            const int r0 = y0 - yb, r1 = y1 + 1 - yb;
            atomicAdd(&cells[r0 * W + x0], 1);
            if (x1 + 1 < W) atomicAdd(&cells[r0 * W + x1 + 1], -1);
            if (r1 < rows) {
                atomicAdd(&cells[r1 * W + x0], -1);
                if (x1 + 1 < W) atomicAdd(&cells[r1 * W + x1 + 1], 1);
            }
        }
        __syncthreads();
        for (int r = wave; r < rows; r += kWaves) {
            int carry = 0;
            for (int x0 = 0; x0 < W; x0 += kWave) {
                const int x = x0 + lane;
                const int v = wave_inclusive_scan(x < W ? cells[r * W + x] : 0) + carry;
                if (x < W) cells[r * W + x] = v;
                carry = __shfl(v, kWave - 1, kWave);
            }
        }
        __syncthreads();
        for (int x = wave; x < W; x += kWaves) {
            int carry = 0;
            for (int r0 = 0; r0 < rows; r0 += kWave) {
                const int r = r0 + lane;
                const int v = wave_inclusive_scan(r < rows ? cells[r * W + x] : 0) + carry;
                if (r < rows) cells[r * W + x] = v;
                carry = __shfl(v, kWave - 1, kWave);
            }
        }
        __syncthreads();
        const int64_t t0 = toff + (int64_t)yb * W;
        for (int i = threadIdx.x; i < n; i += kCountBlock) {
            const int v = cells[i];
            big_len[t0 + i] = v;
            if (v) cnt[t0 + i] += v;
        }
        __syncthreads();   // the next band clears the cells
    }
}

constexpr int kMergeBlock = 256;
constexpr int kMergeWaves = kMergeBlock / kWave;   // tiles per block, one per wave
constexpr int kMergeRing = 512;     // small entries (rank, slot) a wave holds in LDS, as a ring
constexpr int kMergeFill = 256;     // small entries one refill stages
constexpr int kMergeUnroll = 4;     // chunks of big splats whose loads are issued together
constexpr int kMergeLoop = 16;      // groups of up to this many small entries: one ballot per entry

// The LDS of one merge wave: the ring of staged small entries, and for a group of more than
// kMergeLoop small entries, the chunk's big ranks and the group's small ranks.
struct MergeLds {
    int2 ring[kMergeRing];   // small entry i (rank, slot) at i mod kMergeRing
    int32_t big[kWave];
    int32_t grp[kWave];
};

// Stages the small entries [w_hi, w_hi + kMergeFill) below na: ranks from the tile's small
// run A, slots from rank_ids. Called only when w_hi < na and w_hi - p < kWave (p: entries
// placed), so the staged entries not yet placed, at most kWave + kMergeFill <= kMergeRing,
// stay in the ring.
__device__ __forceinline__ void merge_fill(MergeLds &L, const int32_t *__restrict__ A, const int32_t *__restrict__ rank_ids,
                                  int64_t V, int na, int &w_hi)
{
    constexpr int kPer = kMergeFill / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    int32_t r[kPer], s[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) r[u] = A[min(w_hi + u * kWave + lane, na - 1)];   // w_hi < na
#pragma unroll
    for (int u = 0; u < kPer; ++u) s[u] = rank_ids[(int64_t)(uint32_t)r[u] < V ? r[u] : 0];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = w_hi + u * kWave + lane;
        if (i < na) L.ring[i & (kMergeRing - 1)] = make_int2(r[u], s[u]);
    }
    w_hi = min(na, w_hi + kMergeFill);
    __builtin_amdgcn_wave_barrier();
}

// Count of the values of an ascending array of kWave below x (binary lifting over 0 .. 62,
// then entry q itself).
__device__ __forceinline__ int count_below64(const int32_t *arr, int32_t x)
{
    int q = 0;
#pragma unroll
    for (int step = kWave / 2; step > 0; step >>= 1) q = arr[q + step - 1] < x ? q + step : q;
    return arr[q] < x ? q + 1 : q;
}

// Writes entry `at` of a tile's range (ids and keys64 point at its start; below n, its
// length, always when the counts agree).
__device__ inline void put_entry(int at, int n, int32_t id, int t, int32_t *__restrict__ ids,
                                 uint64_t *__restrict__ keys64, const float *__restrict__ depth, int64_t n_splats)
{
    if (at >= n) return;
    ids[at] = id;
    if (keys64)
        keys64[at] = ((uint64_t)(uint32_t)t << 32) |
                     (uint64_t)((uint64_t)(uint32_t)id < (uint64_t)n_splats ? __float_as_uint(depth[id]) : 0u);
}

// The walk of merge_kernel for one tile.
__device__ __forceinline__ void merge_walk(MergeLds &L, const int32_t *__restrict__ A, int na, int t, int tx, int ty,
                                  int n, int64_t b0, int n_cam,
                                  const int4 *__restrict__ big_rec, const int32_t *__restrict__ rank_ids, int64_t V,
                                  int32_t *__restrict__ ids, uint64_t *__restrict__ keys64,
                                  const float *__restrict__ depth, int64_t n_splats, int nb,
                                  int64_t *__restrict__ err_flag)
{
    const int lane = threadIdx.x & (kWave - 1);
    int j = 0;      // contained big splats placed so far
    int p = 0;      // small entries placed so far
    int w_hi = 0;   // small entries staged so far (p <= w_hi)
    const int n_chunks = (n_cam + kWave - 1) / kWave;
    for (int c0 = 0; c0 < n_chunks; c0 += kMergeUnroll) {
        // every load of the group issued before any is used
        int4 rec[kMergeUnroll];
#pragma unroll
        for (int u = 0; u < kMergeUnroll; ++u) rec[u] = big_rec[b0 + min((c0 + u) * kWave + lane, n_cam - 1)];
        bool in[kMergeUnroll];
        int32_t rk[kMergeUnroll], sl[kMergeUnroll];
#pragma unroll
        for (int u = 0; u < kMergeUnroll; ++u) {
            const bool ok = (c0 + u) * kWave + lane < n_cam;
            in[u] = ok & box_holds(make_uint2((uint32_t)rec[u].z, (uint32_t)rec[u].w), tx, ty);
            rk[u] = ok ? rec[u].x : INT32_MAX;
            sl[u] = rec[u].y;
        }
#pragma unroll
        for (int u = 0; u < kMergeUnroll; ++u) {
            if (c0 + u >= n_chunks) break;   // uniform
            const uint64_t m = __ballot(in[u]);
            const int last_lane = min(n_cam - 1 - (c0 + u) * kWave, kWave - 1);
            const int32_t hi = __builtin_amdgcn_readlane(rk[u], last_lane);   // the chunk's last rank
            const int p0 = p;
            int below = 0;   // small entries placed with this chunk that rank below rk[u]
            bool big_staged = false;
            while (p < na) {   // wave-uniform: the next small entries below hi, kWave at a time
                if (w_hi < na && w_hi < p + kWave) merge_fill(L, A, rank_ids, V, na, w_hi);
                const int i = p + lane;
                const int2 e = i < na ? L.ring[i & (kMergeRing - 1)] : make_int2(INT32_MAX, 0);
                const bool here = e.x < hi;   // lanes 0 .. cnt - 1 (the run ascends)
                const int cnt = __popcll(__ballot(here));
                if (cnt == 0) break;
                int q = 0;   // of a small lane: the contained big splats of this chunk below it
                if (cnt <= kMergeLoop) {   // uniform: one ballot per small entry
                    for (int s = 0; s < cnt; ++s) {
                        const int32_t vs = __builtin_amdgcn_readlane(e.x, s);
                        const bool gt = rk[u] > vs;   // ranks are distinct; INT32_MAX past the last
                        below += gt;
                        const int qs = __popcll(m & ~__ballot(gt));
                        q = lane == s ? qs : q;
                    }
                } else {   // binary lifting, each side over the other's ranks in LDS
                    if (!big_staged) {
                        L.big[lane] = rk[u];   // ascending; INT32_MAX past the camera's last big splat
                        big_staged = true;
                    }
                    L.grp[lane] = here ? e.x : INT32_MAX;
                    __builtin_amdgcn_wave_barrier();
                    below += count_below64(L.grp, rk[u]);
                    if (here) q = __popcll(m & ((1ull << count_below64(L.big, e.x)) - 1));   // below hi: < 64
                    __builtin_amdgcn_wave_barrier();   // grp is rewritten by the next group
                }
                if (here) put_entry(i + j + q, n, e.y, t, ids, keys64, depth, n_splats);
                p += cnt;
                if (cnt < kWave) break;
            }
            if (in[u]) put_entry(p0 + below + j + __popcll(m & lanemask_lt()), n, sl[u], t, ids, keys64, depth,
                                 n_splats);
            j += __popcll(m);
        }
    }
    // the rest of the small run lies above every big rank
    for (; p < na; p += kWave) {
        if (w_hi < na && w_hi < p + kWave) merge_fill(L, A, rank_ids, V, na, w_hi);
        const int i = p + lane;
        if (i < na) put_entry(i + j, n, L.ring[i & (kMergeRing - 1)].y, t, ids, keys64, depth, n_splats);
    }
    if (lane == 0 && j != nb)   // unreachable: big_len counted the same boxes
        __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave per tile: its list is the merge, by depth rank, of its small run (the tile-sorted
// small entries, ranks, at svals[ranges[t].start - big_before[t]]) and its big run (its
// camera's big splats whose box contains the tile, in rank order); ranks are distinct. The
// wave walks its camera's big splats in rank order, 64 at a time (one per lane). Per such
// chunk, the small entries not yet placed that rank below the chunk's last rank (the next
// ones of the small run, found by a ballot, up to 64 at a time) are placed: entry i goes to
// start + i + (contained big splats of earlier chunks) + (those of this chunk below it), and
// each big lane counts those below its rank; then a contained big splat goes to start +
// (small entries below it) + (contained big splats before it). What is left of the small
// run after the last chunk lies above every big rank. The small run passes through a ring in
// the wave's LDS, with each entry's slot fetched when it is staged. Entry = slot; the key
// (tile << 32 | depth bits) only when asked for. No block barriers: the waves share nothing.
__global__ __launch_bounds__(kMergeBlock) void merge_kernel(const gs_camera *__restrict__ cams, int n_cams,
                                                            int n_tiles, const int64_t *__restrict__ words,
                                                            const int32_t *__restrict__ ranges,
                                                            const int32_t *__restrict__ big_len,
                                                            const int32_t *__restrict__ big_before,
                                                            const int4 *__restrict__ big_rec,
                                                            const int32_t *__restrict__ svals,
                                                            const int32_t *__restrict__ rank_ids,
                                                            const int64_t *__restrict__ vcount,
                                                            int32_t *__restrict__ ids, uint64_t *__restrict__ keys64,
                                                            const float *__restrict__ depth, int64_t n_splats,
                                                            int64_t *__restrict__ err_flag)
{
    __shared__ MergeLds lds[kMergeWaves];
    if (!words[kBigOk] || *err_flag) return;   // uniform
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));   // uniform: scalar tile state
    const int t = (int)(blockIdx.x * kMergeWaves + wave);
    if (t >= n_tiles) return;   // wave-uniform; the waves of a block share no barrier
    const int64_t start = ranges[2 * t], n = (int64_t)ranges[2 * t + 1] - start;
    if (n <= 0) return;
    const int nb = big_len[t], na = (int)n - nb;
    const int64_t k_small = words[kBigEffSmall], V = *vcount;
    const int64_t ss = start - big_before[t];
    if (na < 0 || ss < 0 || ss + na > k_small) {   // unreachable when the counts agree
        if ((threadIdx.x & (kWave - 1)) == 0)
            __hip_atomic_store(err_flag, (int64_t)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int cam = camera_of_tile(cams, n_cams, t);
    const int local = t - cams[cam].tile_offset, tw = max(cams[cam].tiles_x, 1), tx = local % tw, ty = local / tw;
    const int64_t b0 = words[kBigCamStart + cam];
    const int n_cam = (int)(words[kBigCamStart + cam + 1] - b0);
    merge_walk(lds[wave], svals + ss, na, t, tx, ty, (int)n, b0, n_cam, big_rec, rank_ids, V, ids + start,
               keys64 ? keys64 + start : keys64, depth, n_splats, nb, err_flag);
}

// Zeroes a[0, na) and b[0, nb) in one launch (grid-stride; consecutive threads take
// consecutive words), and the work-list header except its walk stamp.
__global__ __launch_bounds__(256) void zero_pair_kernel(int32_t *__restrict__ a, int64_t na, int32_t *__restrict__ b,
                                                        int64_t nb, int32_t *__restrict__ sched)
{
    const int64_t n = na + nb, step = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (first < kSchedHeader && first != kSchedWalkStamp) sched[first] = 0;
    for (int64_t i = first; i < n; i += step) {
        if (i < na) a[i] = 0;
        else b[i - na] = 0;
    }
}

// chunk_rank[c] = depth rank of the splat that holds list entry c * kSortChunk
// (rank_tiles: tiles_touched in rank order).
__global__ __launch_bounds__(256) void chunk_rank_kernel(const int32_t *__restrict__ rank_ids,
                                                         const int64_t *__restrict__ offsets,
                                                         const int32_t *__restrict__ rank_tiles,
                                                         const int64_t *__restrict__ vcount,
                                                         const int64_t *__restrict__ count, int64_t cap,
                                                         int32_t *__restrict__ chunk_rank,
                                                         const int64_t *__restrict__ err_flag)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (*err_flag || r >= *vcount) return;
    const int n = rank_tiles[r];
    if (n <= 0) return;
    const int64_t kvalid = tile_sort_count(count, cap);
    const int64_t s = offsets[r], e = s + n;
    for (int64_t c = (s + kSortChunk - 1) / kSortChunk; c * kSortChunk < e && c * kSortChunk < kvalid; ++c)
        chunk_rank[c] = (int32_t)r;
}

// ------------------------------------------------------------------------ work list

__device__ inline int length_bucket(int len)
{
    // bucket 0 holds the longest lists; empty tiles land in the last bucket
    const int lg = 31 - __clz(len + 1);
    return kSchedNumBuckets - 1 - min(kSchedNumBuckets - 1, lg);
}

// Clears the header, except the walk-length stamp.
// The length a tile is scheduled by: its list length, or the walk length of the last
// rasterization when recorded for this tile count (and not longer than the list).
__device__ inline int sched_len(const int32_t *__restrict__ ranges, const int32_t *__restrict__ sched, int n_tiles,
                                int t)
{
    const int len = ranges[2 * t + 1] - ranges[2 * t];
    if (len <= 0 || sched[kSchedWalkStamp] != n_tiles) return len;
    const int walk = sched[sched_walk_offset(n_tiles) + t];
    return walk >= 1 && walk < len ? walk : len;
}

// Per-block bucket histogram in LDS, then one global atomic per non-empty bucket (the header
// was zeroed at the start of the call). When the sort's error word is set (a wait gave up, or
// the counts disagree) the ranges are emptied first, whatever wrote them, so nothing reads
// the list, and the word joins the flags (2: the list is invalid; 4: a camera wider than the
// count array).
__global__ __launch_bounds__(256) void sched_count_kernel(int32_t *__restrict__ ranges, int n_tiles, int split_len,
                                                          int split_items, int32_t *__restrict__ sched,
                                                          const int64_t *__restrict__ err,
                                                          int64_t *__restrict__ counters)
{
    __shared__ int cnt[kSchedNumBuckets];
    if (threadIdx.x < kSchedNumBuckets) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0 && err && *err) counters[1] |= *err;
    if (t < n_tiles) {
        if (err && *err) ranges[2 * t] = ranges[2 * t + 1] = 0;
        const int len = sched_len(ranges, sched, n_tiles, t);
        atomicAdd(&cnt[length_bucket(len)], len >= split_len ? split_items : 1);
    }
    __syncthreads();
    if (threadIdx.x < kSchedNumBuckets && cnt[threadIdx.x])
        atomicAdd(&sched[kSchedBuckets + threadIdx.x], cnt[threadIdx.x]);
}

// Each block reserves one contiguous run per bucket (one global atomic per bucket), then
// hands out positions inside its runs with LDS atomics. Order inside a bucket is free.
__global__ __launch_bounds__(256) void sched_fill_kernel(const int32_t *__restrict__ ranges, int n_tiles,
                                                         int split_len, int split_parts, int bwd_segs,
                                                         int32_t *__restrict__ sched)
{
    __shared__ int cnt[kSchedNumBuckets], base[kSchedNumBuckets];
    if (threadIdx.x < kSchedNumBuckets) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int len = 0, b = 0, n = 0;
    if (t < n_tiles) {
        len = sched_len(ranges, sched, n_tiles, t);
        b = length_bucket(len);
        n = len >= split_len ? split_parts * bwd_segs : 1;
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
            sched[kSchedSegs] = bwd_segs;
        }
    }
    __syncthreads();
    if (t >= n_tiles) return;
    const int pos = base[b] + atomicAdd(&cnt[b], n);
    int32_t *items = sched + kSchedHeader;
    if (n == 1) {
        items[pos] = t << kItemTileShift;
    } else {
        // segment-major, so that the parts of one segment start together
        for (int seg = 0; seg < bwd_segs; ++seg)
            for (int part = 0; part < split_parts; ++part)
                items[pos + seg * split_parts + part] = (t << kItemTileShift) | (seg << 3) | 4 | part;
    }
}

// ------------------------------------------------------------------------ workspace

// Workspace: depth-sort buffers (two key/value pairs over P splats; the last depth pass
// leaves the tile counts in rank order where the keys were), the visible count, per-rank
// emit offsets, per-chunk counts and sums of the two scans, one 32-bit key/value pair over
// the capacity (the other pair of the tile-sort ping-pong lives in bins->keys / bins->ids
// until the last pass overwrites them), then a region cleared at the start of every call:
// the per-tile difference array (then list lengths), the look-back status words of the
// ranges scan and of every sort pass, the digit histograms and an error word.
constexpr int kMaxTilePasses = 4;

struct BinLayout {
    size_t dkeyA, dvalA, dkeyB, dvalB, dcount, offsets, chunk_cnt, chunk_sum, tkey, tval, chunk_rank;
    size_t big_mat, big_rec, big_len, big_before;
    size_t zero_begin, gdiff, stat_ranges, stat_depth, stat_tile, ghist_depth, ghist_tile;
    size_t big_words, err;
    size_t total;
    int64_t depth_nb, tile_nb, big_cap;
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
    L.chunk_cnt = o;   o += align256((size_t)L.depth_nb * sizeof(int32_t));
    L.chunk_sum = o;   o += align256((size_t)L.depth_nb * sizeof(int64_t));
    L.tkey = o;        o += align256((size_t)cap * 4);
    L.tval = o;        o += align256((size_t)cap * 4);
    L.chunk_rank = o;  o += align256((size_t)(L.tile_nb + 1) * sizeof(int32_t));
    // splats listed by the merge: each adds more than kBigMinTiles entries to a list that fits
    L.big_cap = min(n_splats, cap / (kBigMinTiles + 1));
    L.big_mat = o;     o += align256((size_t)L.depth_nb * kBigMaxCams * sizeof(int32_t));
    L.big_rec = o;     o += align256((size_t)L.big_cap * sizeof(int4));
    L.big_len = o;     o += align256((size_t)n_tiles * sizeof(int32_t));
    L.big_before = o;  o += align256((size_t)n_tiles * sizeof(int32_t));
    L.zero_begin = o;
    L.gdiff = o;       o += align256((size_t)n_tiles * sizeof(int32_t));
    L.stat_ranges = o; o += align256((size_t)((n_tiles + kSortChunk - 1) / kSortChunk) * sizeof(uint64_t));
    L.stat_depth = o;  o += align256((size_t)kDepthPasses * L.depth_nb * stat_row);
    L.stat_tile = o;   o += align256((size_t)L.tile_passes * L.tile_nb * stat_row);
    L.ghist_depth = o; o += align256((size_t)kDepthPasses * kRadix * sizeof(unsigned));
    L.ghist_tile = o;  o += align256((size_t)kMaxTilePasses * kRadix * sizeof(unsigned));
    L.big_words = o;   o += align256((size_t)kBigWords * sizeof(int64_t));
    L.err = o;         o += 256;
    L.total = o;
    return L;
}

// Grid of a single-pass launch whose blocks wait on each other (chunk_stop): no more blocks
// than the device holds at once for this kernel (its occupancy per CU, at most four), so
// every block is resident and every wait ends; never more blocks than chunks.
static unsigned resident_grid(const void *kernel, int block, int64_t chunks)
{
    struct Entry {
        const void *k;
        int dev, per_cu;
    };
    static std::mutex mu;
    static Entry cache[32];
    static int n_cache = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (int i = 0; i < n_cache; ++i)
            if (cache[i].k == kernel && cache[i].dev == dev) per_cu = cache[i].per_cu;
        if (per_cu == 0) {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1) {
                (void)hipGetLastError();
                per_cu = 1;
            }
            per_cu = min(per_cu, 4);
            if (n_cache < 32) cache[n_cache++] = Entry{kernel, dev, per_cu};
        }
    }
    const int64_t g = (int64_t)device_cu_count() * per_cu;
    return (unsigned)max((int64_t)1, min(g, chunks));
}

}  // namespace gsx

using namespace gsx;

// The work list (its header was zeroed at the start of the call); the sort's error word
// joins the flags.
static int build_schedule(gs_bins *bins, const int64_t *err, hipStream_t st)
{
    const unsigned g = grid_for(bins->n_tiles, 256);
    const gs_tuning &tu = current_tuning();
    hipLaunchKernelGGL(sched_count_kernel, dim3(g), dim3(256), 0, st, bins->ranges, bins->n_tiles, tu.split_len,
                       tu.split_parts * tu.bwd_segs, bins->schedule, err, bins->counters);
    hipLaunchKernelGGL(sched_fill_kernel, dim3(g), dim3(256), 0, st, bins->ranges, bins->n_tiles, tu.split_len,
                       tu.split_parts, tu.bwd_segs, bins->schedule);
    return check_launch("gs_bin_and_sort");
}

extern "C" int64_t gs_schedule_size(int32_t n_tiles)
{
    return n_tiles < 0 ? 0 : sched_walk_offset(n_tiles) + n_tiles;
}

extern "C" size_t gs_bin_and_sort_workspace_size(int64_t n_splats, int64_t capacity, int32_t n_tiles)
{
    if (n_splats < 0 || capacity < 1 || n_tiles < 1) return 0;
    return bin_layout(n_splats, capacity, n_tiles).total;
}

// Argument checks shared by the entry points of binning.
static int check_bin_args(const gs_splats *s, int64_t n_splats, const gs_camera *cams, int32_t n_cams,
                          const gs_bins *bins)
{
    if (!s || !cams || !bins || n_cams < 1 || n_splats < 0)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: null argument or bad size");
    if (bins->capacity < 1 || bins->capacity > 0x7fffffffll || bins->n_tiles < 1)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: capacity must be in [1, 2^31-1], n_tiles >= 1");
    if (n_splats > 0x7fffffffll)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: n_splats must be below 2^31");
    if (n_cams > bins->n_tiles)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: more cameras than tiles");
    if (bins->flags & ~GS_BINS_NO_KEYS)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: unknown bits in flags");
    if (!bins->keys || !bins->ids || !bins->ranges || !bins->schedule || !bins->counters || !s->rect || !s->depth ||
        !s->tiles_touched || n_splats > s->capacity)
        return set_error(GS_ERR_INVALID, "gs_bin_and_sort: null buffer or n_splats > capacity");
    return GS_OK;
}

// The launches of one call, on the workspace ws (layout L, 256-byte aligned); every part of
// ws that must start at zero is cleared by the call's first launch.
static int bin_and_sort_run(const gs_splats *s, int64_t n_splats, const gs_camera *cams, int32_t n_cams,
                            gs_bins *bins, char *ws, const BinLayout &L, hipStream_t st)
{
    const int64_t cap = bins->capacity;
    uint32_t *dkeyA = (uint32_t *)(ws + L.dkeyA), *dkeyB = (uint32_t *)(ws + L.dkeyB);
    int32_t *dvalA = (int32_t *)(ws + L.dvalA), *dvalB = (int32_t *)(ws + L.dvalB);
    int64_t *dcount = (int64_t *)(ws + L.dcount);
    int64_t *offsets = (int64_t *)(ws + L.offsets);
    int32_t *tile_cnt = (int32_t *)(ws + L.gdiff);
    int32_t *chunk_cnt = (int32_t *)(ws + L.chunk_cnt);
    int64_t *chunk_sum = (int64_t *)(ws + L.chunk_sum);
    uint64_t *stat_ranges = (uint64_t *)(ws + L.stat_ranges);
    uint64_t *stat_depth = (uint64_t *)(ws + L.stat_depth), *stat_tile = (uint64_t *)(ws + L.stat_tile);
    unsigned *ghist_depth = (unsigned *)(ws + L.ghist_depth), *ghist_tile = (unsigned *)(ws + L.ghist_tile);
    int64_t *err = (int64_t *)(ws + L.err);
    const int64_t *K = (const int64_t *)bins->counters;
    // splats with more than big_tiles tiles are listed by the per-tile merge (launch tuning;
    // calls with more cameras than the merge's table take the plain sort)
    const int big_tiles = (current_tuning().big_tiles > 0 && n_cams <= kBigMaxCams) ? current_tuning().big_tiles : 0;
    int32_t *big_mat = (int32_t *)(ws + L.big_mat);
    int4 *big_rec = (int4 *)(ws + L.big_rec);
    int32_t *big_len = (int32_t *)(ws + L.big_len), *big_before = (int32_t *)(ws + L.big_before);
    int64_t *big_words = (int64_t *)(ws + L.big_words);

    // ranges start empty, (0, 0); the look-back state, counts, histograms and the work-list header start at zero
    if (n_splats == 0) {
        hipLaunchKernelGGL(zero_pair_kernel, dim3(grid_for(2ll * bins->n_tiles, 256)), dim3(256), 0, st,
                           bins->ranges, 2ll * bins->n_tiles, (int32_t *)bins->counters, (int64_t)4, bins->schedule);
        return build_schedule(bins, (const int64_t *)nullptr, st);
    }
    {
        const int64_t nz = (int64_t)((L.total - L.zero_begin) / 4), n = 2ll * bins->n_tiles + nz;
        hipLaunchKernelGGL(zero_pair_kernel, dim3((unsigned)min(grid_for(n, 256), 4096u)), dim3(256), 0, st,
                           bins->ranges, 2ll * bins->n_tiles, (int32_t *)(ws + L.zero_begin), nz, bins->schedule);
    }
    int rc = GS_OK;

    // 1. the V visible splats, compacted in slot order, with the digit counts of the depth
    // passes; the list length of every tile from their boxes, and the digit counts of the
    // tile passes from those
    const int passes = L.tile_passes;
    // launches without waits between blocks take one block per chunk
    const unsigned g_chunks = (unsigned)L.depth_nb;
    const unsigned g_sort = resident_grid((const void *)onesweep_kernel, kSortBlock, L.depth_nb);
    hipLaunchKernelGGL(visible_count_kernel, dim3(g_chunks), dim3(kSortBlock), 0, st, s->tiles_touched, n_splats,
                       chunk_cnt);
    hipLaunchKernelGGL(chunk_scan_kernel<int32_t>, dim3(1), dim3(kScanBlock), 0, st, chunk_cnt, n_splats,
                       (const int64_t *)nullptr, dcount, (int64_t *)nullptr, (int64_t)0);
    hipLaunchKernelGGL(visible_write_kernel, dim3(g_chunks), dim3(kSortBlock), 0, st, s->tiles_touched, s->depth,
                       n_splats, (const int32_t *)chunk_cnt, dkeyA, dvalA);
    hipLaunchKernelGGL(depth_hist_kernel, dim3((unsigned)min(L.depth_nb, (int64_t)device_cu_count() * 2)),
                       dim3(kSortBlock), 0, st, (const uint32_t *)dkeyA, (const int64_t *)dcount, ghist_depth);
    const int64_t span = max((int64_t)8192, (n_splats + 511) / 512);
    hipLaunchKernelGGL(tile_corner_kernel, dim3(grid_for(n_splats, (int)span)), dim3(kCornerBlock), 0, st,
                       (const int32_t *)dvalA, (const int64_t *)dcount, (const int4 *)s->rect, cams, (int)n_cams,
                       n_splats, span, big_tiles, tile_cnt);
    hipLaunchKernelGGL(tile_count_kernel, dim3((unsigned)n_cams), dim3(kCountBlock), 0, st, cams, passes, tile_cnt,
                       ghist_tile, err);

    // 2. depth order: four 8-bit passes over the V keys (the result is back in A; the last
    // pass writes the tile counts in rank order over the keys, which are not needed)
    static_assert(kDepthPasses % 2 == 0, "the depth passes end in A");
    int32_t *rank_tiles = (int32_t *)dkeyA;
    for (int pass = 0; pass < kDepthPasses; ++pass) {
        const bool even = (pass & 1) == 0, last = pass == kDepthPasses - 1;
        hipLaunchKernelGGL(onesweep_kernel, dim3(g_sort), dim3(kSortBlock), 0, st, even ? dkeyA : dkeyB,
                           even ? dvalA : dvalB, (const int64_t *)dcount, n_splats, pass * kRadixBits,
                           ghist_depth + pass * kRadix, stat_depth + (int64_t)pass * L.depth_nb * kRadix,
                           last ? (uint32_t *)nullptr : (even ? dkeyB : dkeyA), even ? dvalB : dvalA,
                           (uint64_t *)nullptr, (const float *)nullptr,
                           last ? (const int32_t *)s->tiles_touched : (const int32_t *)nullptr,
                           last ? rank_tiles : (int32_t *)nullptr, n_splats, 0, err);
    }
    rc = check_launch("depth sort");
    if (rc != GS_OK) return rc;
    const int32_t *rank_ids = dvalA;

    // 3. emit offsets in depth-rank order; K and the overflow flag go to bins->counters
    hipLaunchKernelGGL(rank_sum_kernel, dim3(g_chunks), dim3(kSortBlock), 0, st, (const int32_t *)rank_tiles,
                       (const int64_t *)dcount, chunk_sum, big_tiles);
    // with the merge, the scan gives the entries of small splats; big_scan then sets K
    hipLaunchKernelGGL(chunk_scan_kernel<int64_t>, dim3(1), dim3(kScanBlock), 0, st, chunk_sum, (int64_t)0,
                       (const int64_t *)dcount, big_tiles ? big_words + kBigKSmall : bins->counters,
                       big_tiles ? (int64_t *)nullptr : bins->counters + 1, cap);
    hipLaunchKernelGGL(rank_offsets_kernel, dim3(g_chunks), dim3(kSortBlock), 0, st, (const int32_t *)rank_tiles,
                       (const int64_t *)dcount, (const int64_t *)chunk_sum, offsets, big_tiles);
    if (big_tiles) {
        hipLaunchKernelGGL(big_count_kernel, dim3(g_chunks), dim3(kSortBlock), 0, st, rank_ids,
                           (const int32_t *)rank_tiles, (const int64_t *)dcount, cams, (int)n_cams, big_tiles, big_mat,
                           L.depth_nb, big_words, (const int64_t *)err);
        hipLaunchKernelGGL(big_scan_kernel, dim3((unsigned)n_cams), dim3(kScanBlock), 0, st, big_mat, L.depth_nb,
                           (const int64_t *)dcount, (int)n_cams, big_words, bins->counters, cap, L.big_cap, err);
        hipLaunchKernelGGL(big_scatter_kernel, dim3(g_chunks), dim3(kSortBlock), 0, st, rank_ids,
                           (const int32_t *)rank_tiles, (const int64_t *)dcount, cams, (int)n_cams, big_tiles,
                           (const int4 *)s->rect, (const int32_t *)big_mat, L.depth_nb, (const int64_t *)big_words,
                           big_rec, err);
    }
    // entries the tile passes sort: all K (or none on overflow), or the small splats' ones
    const int64_t *sort_n = big_tiles ? (const int64_t *)(big_words + kBigEffSmall) : K;

    // 4. stable passes by tile id. The first pass takes the entries in depth-rank order,
    // either emitted into a buffer or generated inside the pass (launch tuning); the last
    // reads the workspace pair W and writes bins; in between, passes alternate between W
    // and the pair stored in bins' buffers.
    const unsigned g_tile = resident_grid((const void *)onesweep_kernel, kSortBlock, L.tile_nb);
    uint32_t *kW = (uint32_t *)(ws + L.tkey), *kX = (uint32_t *)bins->keys;
    int32_t *vW = (int32_t *)(ws + L.tval), *vX = bins->ids;
    // the sorted 64-bit keys, unless the caller does without them (the last pass then writes
    // ids only and gathers no depth)
    uint64_t *keys_final = (bins->flags & GS_BINS_NO_KEYS) ? (uint64_t *)nullptr : bins->keys;
    // Without the merge the last pass writes the list (ids, keys) into bins; with it, the
    // last pass writes tile keys and ranks into W, which the merge reads. Pass i writes the
    // pair the last pass writes when (passes - 1 - i) is even, the other pair otherwise.
    const bool first_to_W = big_tiles ? ((passes - 1) & 1) == 0 : passes >= 2 && ((passes - 2) & 1) == 0;
    // (with the merge, the last pass writes only the ranks: nothing reads its tile keys)
    uint32_t *k0out = passes == 1 ? (uint32_t *)nullptr : (first_to_W ? kW : kX);
    int32_t *v0out = passes == 1 && !big_tiles ? bins->ids : (first_to_W ? vW : vX);
    uint64_t *k64 = passes == 1 && !big_tiles ? keys_final : (uint64_t *)nullptr;
    if (current_tuning().generate_entries && !big_tiles) {
        int32_t *chunk_rank = (int32_t *)(ws + L.chunk_rank);
        hipLaunchKernelGGL(chunk_rank_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, st, rank_ids, offsets,
                           (const int32_t *)rank_tiles, (const int64_t *)dcount, K, cap, chunk_rank,
                           (const int64_t *)err);
        hipLaunchKernelGGL(onesweep_emit_kernel,
                           dim3(resident_grid((const void *)onesweep_emit_kernel, kSortBlock, L.tile_nb)),
                           dim3(kSortBlock), 0, st, rank_ids, offsets, (const int32_t *)chunk_rank,
                           (const int32_t *)rank_tiles,
                           (const int4 *)s->rect, cams, (int)n_cams, n_splats, (const int64_t *)dcount, K, cap,
                           ghist_tile, stat_tile, k0out, v0out, k64, s->depth, err);
    } else {
        // the emitted entries go to the pair the first pass does not write
        const bool emit_to_X = big_tiles ? first_to_W : passes >= 2 && first_to_W;
        uint32_t *ek = emit_to_X ? kX : kW;
        int32_t *ev = emit_to_X ? vX : vW;
        hipLaunchKernelGGL(emit_kernel, dim3(min(grid_for(n_splats, 256), (unsigned)device_cu_count() * 8)), dim3(256),
                           0, st, rank_ids, offsets,
                           (const int32_t *)rank_tiles, (const int4 *)s->rect, cams, (int)n_cams, n_splats,
                           (const int64_t *)dcount, K, cap, ek, ev, big_tiles, (const int64_t *)err);
        hipLaunchKernelGGL(onesweep_kernel, dim3(g_tile), dim3(kSortBlock), 0, st, ek, ev, sort_n, cap, 0, ghist_tile,
                           stat_tile, k0out, v0out, k64, s->depth, (const int32_t *)nullptr, (int32_t *)nullptr,
                           n_splats, 1, err);
    }
    uint32_t *kin = first_to_W ? kW : kX;
    int32_t *vin = first_to_W ? vW : vX;
    for (int pass = 1; pass < passes; ++pass) {
        const bool last = pass == passes - 1 && !big_tiles;
        uint32_t *kout = kin == kW ? kX : kW;
        int32_t *vout = vin == vW ? vX : vW;
        hipLaunchKernelGGL(onesweep_kernel, dim3(g_tile), dim3(kSortBlock), 0, st, kin, vin, sort_n, cap,
                           pass * kRadixBits, ghist_tile + pass * kRadix,
                           stat_tile + (int64_t)pass * L.tile_nb * kRadix,
                           pass == passes - 1 ? (uint32_t *)nullptr : kout,
                           last ? bins->ids : vout,
                           last ? keys_final : (uint64_t *)nullptr, s->depth, (const int32_t *)nullptr,
                           (int32_t *)nullptr, n_splats, 1, err);
        kin = kout;
        vin = vout;
    }
    rc = check_launch("tile sort");
    if (rc != GS_OK) return rc;
    if (big_tiles)   // the big splats' tiles join the list lengths
        hipLaunchKernelGGL(big_len_kernel, dim3((unsigned)n_cams), dim3(kCountBlock), 0, st, cams, (int)n_cams,
                           (const int64_t *)big_words, (const int4 *)big_rec, tile_cnt, big_len,
                           (const int64_t *)err);
    // 5. ranges from the list lengths, when the list was built
    hipLaunchKernelGGL(ranges_kernel,
                       dim3(resident_grid((const void *)ranges_kernel, kSortBlock, grid_for(bins->n_tiles, kSortChunk))),
                       dim3(kSortBlock), 0, st, (const int32_t *)tile_cnt, bins->n_tiles, K, cap, stat_ranges,
                       bins->ranges, big_tiles ? (const int32_t *)big_len : (const int32_t *)nullptr,
                       big_tiles ? big_before : (int32_t *)nullptr, err);
    if (big_tiles) {   // the small run (sorted into W) and the big run of each tile, merged into bins
        hipLaunchKernelGGL(merge_kernel, dim3(grid_for(bins->n_tiles, kMergeWaves)), dim3(kMergeBlock), 0, st, cams,
                           (int)n_cams,
                           bins->n_tiles, (const int64_t *)big_words, (const int32_t *)bins->ranges,
                           (const int32_t *)big_len, (const int32_t *)big_before, (const int4 *)big_rec,
                           (const int32_t *)vW, rank_ids,
                           (const int64_t *)dcount, bins->ids, keys_final, s->depth, n_splats, err);
        rc = check_launch("merge");
        if (rc != GS_OK) return rc;
    }

    // 6. the work list
    return build_schedule(bins, (const int64_t *)err, st);
}

extern "C" int gs_set_sort_wait_limit(int32_t polls)
{
    clear_error();
    return check_hip(hipMemcpyToSymbol(HIP_SYMBOL(g_wait_limit), &polls, sizeof(polls)), "gs_set_sort_wait_limit");
}

extern "C" int gs_bin_and_sort(const gs_splats *s, int64_t n_splats, const gs_camera *cams, int32_t n_cams,
                               gs_bins *bins, void *workspace, size_t workspace_bytes, void *stream)
{
    clear_error();
    int rc = check_bin_args(s, n_splats, cams, n_cams, bins);
    if (rc != GS_OK) return rc;
    const BinLayout L = bin_layout(n_splats, bins->capacity, bins->n_tiles);
    if (!workspace || workspace_bytes < L.total)
        return set_error(GS_ERR_CAPACITY, "gs_bin_and_sort: workspace too small");
    if (((uintptr_t)workspace) & 255) return set_error(GS_ERR_INVALID, "gs_bin_and_sort: workspace not 256-byte aligned");
    return bin_and_sort_run(s, n_splats, cams, n_cams, bins, (char *)workspace, L, (hipStream_t)stream);
}

// ------------------------------------------------- the variant that allocates nothing

// The workspace of gs_bin_and_sort_static: a file-scope device array, one per GPU, held until
// the process ends. In host code its name is only a stand-in for the symbol; the device
// address comes from hipGetSymbolAddress, once per device, and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[GS_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static int scratch_for_current_device(char **out)
{
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "gs_bin_and_sort_static: hipGetDevice");
    if (rc != GS_OK) return rc;
    if (dev < 0 || dev >= kMaxDevices) return set_error(GS_ERR_DEVICE, "gs_bin_and_sort_static: device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "gs_bin_and_sort_static: hipGetSymbolAddress");
        if (rc != GS_OK) return rc;
        if (!p || (((uintptr_t)p) & 255))
            return set_error(GS_ERR_HIP, "gs_bin_and_sort_static: scratch symbol has no aligned device address");
        g_scratch_ptr[dev] = p;
    }
    *out = (char *)g_scratch_ptr[dev];
    return GS_OK;
}

extern "C" int gs_bin_and_sort_static(const gs_splats *s, int64_t n_splats, const gs_camera *cams, int32_t n_cams,
                                      gs_bins *bins, void *stream)
{
    clear_error();
    int rc = check_bin_args(s, n_splats, cams, n_cams, bins);
    if (rc != GS_OK) return rc;
    const BinLayout L = bin_layout(n_splats, bins->capacity, bins->n_tiles);
    if (L.total > (size_t)GS_STATIC_WORKSPACE_BYTES)
        return set_error(GS_ERR_CAPACITY, "gs_bin_and_sort_static: the call needs more workspace than the library's "
                                          "static GS_STATIC_WORKSPACE_BYTES; use gs_bin_and_sort with a workspace");
    char *ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc != GS_OK) return rc;
    return bin_and_sort_run(s, n_splats, cams, n_cams, bins, ws, L, (hipStream_t)stream);
}
