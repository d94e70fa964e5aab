// gs_rasterize_fwd / gs_rasterize_bwd: per-tile compositing (Sec. 2.2, eq. 7) and its
// gradients (Sec. 3.1, eqs. 16-21).
//
// Work items. gs_bin_and_sort leaves a work list of tiles in decreasing list length
// (longest first). A tile with a short list is one item: one wave64, four horizontally
// adjacent pixels per lane. A tile with a long list (the length threshold and the split
// are launch tuning, gs_tuning) is two 16x8-pixel halves at two pixels per lane or four
// 16x4-pixel quarters at one pixel per lane, so that its walk, the critical path of the
// launch, is split over several waves; in the fused kernel the backward of a split tile can
// also be walked as list segments by separate items (each repeating the forward, which
// snapshots T and the colour at the segment's end). The kernels are persistent: every wave
// takes items from an atomic counter until the list is exhausted, and the last wave out
// resets the counter so the next launch (or graph replay) starts from zero. A wave may raise
// its issue priority (s_setprio) while it works on a split item or a long unsplit tile, in
// levels by walk length, so that the longest walks keep most of their SIMD.
//
// Records. A wave walks its list in batches of 64 entries. For each batch every lane
// gathers one entry's 64-byte RasterRec with vector loads (64 records in flight per wave)
// into registers, one batch ahead, so the random record reads stay off the critical path.
// Each lane then tests its record against the rectangle of the pixel centres of the lanes
// still active (unfinished in the forward, not past their last entry in the backward);
// records that cannot reach alpha_min there are dropped, and the rest are staged packed,
// in list order, into the wave's own LDS slice (the forward pads them to a multiple of 8
// with null records and composites groups of 8 as straight-line code). The walk reads each
// record back with broadcast LDS loads. No workgroup barrier is ever needed: a wave only
// reads the LDS slice it wrote. Per lane and splat the row terms
// lo + C dy^2 and B dy are formed once and shared by the lane's pixels; per pixel the
// exponent costs one subtraction and two FMAs in float64 (exact Delta, no cancellation
// loss), one conversion and a float32 exp2. Compositing is branch-free: a pixel that
// skips, stops or is done composites with weight zero.
//
// Backward: each pixel walks its list from `last` down, recomputing alpha with the same
// instructions as the forward, recovering T = T_after / (1 - alpha) (eq. 17) and carrying
// G_S = sum_k dL/dC(k) S(k) (eq. 18 summed over channels). Per lane it sums the nine
// per-pair terms of its pixels,
//   v = dL/dalpha * alpha, v dx, v dy, v dx^2, v dx dy, v dy^2, alpha T dL/dC(k) (k = 0..2)
// which are summed per splat in an LDS slot (see WaveAcc) and moved to memory with one
// atomic per term and splat at the end of each batch:
//   dL/do = sum v / o, dL/dmu' = -Y sum v Delta, dL/dY = -1/2 sum v Delta Delta^T, dL/dc.
#include "common.h"

namespace gsx {

constexpr int kBlockWaves = 4;
// List entries staged per wave and batch: B = 32 or 64 (launch tuning, gs_tuning.batch; a
// template parameter of the walks). One lane gathers one record, so B <= 64; the LDS slices
// are sized for 64.
constexpr int kBatch = kWave;

// Work counters (gs_set_work_counter): when set, [0] += (list slots a forward walk stepped
// through) x (pixels of its wave), [1] += the same for the backward walks. A measurement aid:
// the counts are the Gaussian-pixel pairs the kernels execute, padding and finished pixels
// included, as opposed to the pairs the method defines.
__constant__ unsigned long long *g_work_count = nullptr;

// The wave's LDS slice for one batch of records.
__device__ inline RasterRec *wave_slice()
{
    __shared__ RasterRec slice[kBlockWaves][kBatch];
    return slice[__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))];
}

// A batch is gathered in two dependent steps, each issued one batch ahead of its use: the
// list entries' splat slots (load_ids), then their 64-byte records (gather) into registers,
// one per lane. The records carry their own slot, so nothing is merged into the loads'
// destination registers while the loads are in flight.
struct Gathered {
    float4 q0, q1, q2, q3;
};

// Splat slots of list entries [b, b + n), one per lane; -1 for lanes >= n.
__device__ inline int load_ids(const int32_t *__restrict__ ids, int b, int n, int lane)
{
    return lane < n ? ids[b + lane] : -1;
}

__device__ inline Gathered gather(const RasterRec *__restrict__ rr, int id)
{
    Gathered g;
    if (id >= 0) {
        const float4 *p = (const float4 *)(rr + id);
        g.q0 = p[0];
        g.q1 = p[1];
        g.q2 = p[2];
        g.q3 = p[3];
    } else {
        g.q0 = g.q1 = g.q2 = g.q3 = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return g;
}

// Entries a walk goes through per group: the walks run over whole groups, the all-finished
// test of the forward is made between groups, and the staged batch is padded to a multiple.
constexpr int kGroup = 8;

// Stages the lanes' gathered records selected by `keep` (a lane mask) into the slice,
// packed in lane order: the record of the k-th selected lane goes to slot k. The staged copy
// carries, in place of o (which the walks do not read), the record's list position plus
// one (p1 of the lane, an int). Slots from the number kept up to the next multiple of kGroup
// receive a null record (alpha 0 at every pixel, colour 0, position 0): a walk step over it
// changes nothing. Returns the number of slots to walk (kept records plus padding).
__device__ inline int stage_packed(RasterRec *slice, const Gathered &g, uint64_t keep, int lane, int p1)
{
    const int nk = __popcll(keep);
    const int np = (nk + kGroup - 1) & ~(kGroup - 1);
    if ((keep >> lane) & 1) {
        const int k = __builtin_amdgcn_mbcnt_hi((unsigned)(keep >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)keep, 0u));
        float4 *d = (float4 *)(slice + k);
        d[0] = g.q0;
        d[1] = g.q1;
        d[2] = g.q2;
        d[3] = make_float4(g.q3.x, __int_as_float(p1), g.q3.z, g.q3.w);
    }
    if (lane >= nk && lane < np) {
        // lo = -1e30 with A = B = C = 0 gives an exponent of -1e30 (finite) and alpha = exp2 = 0
        RasterRec z;
        z.mx = z.my = 0.f;
        z.lo = -1e30;
        z.A = z.B = z.C = 0.0;
        z.c0 = z.c1 = z.c2 = 0.f;
        z.o = __int_as_float(0);
        z.src = z.slot = 0;
        slice[lane] = z;
    }
    return np;
}

// List position plus one of a staged record (stored in place of o); wave-uniform, since every
// lane reads the same slot.
__device__ __forceinline__ int staged_p1(const RasterRec &r)
{
    return __builtin_amdgcn_readfirstlane(__float_as_int(r.o));
}

struct ItemPixels {
    int start, end;
    int row, col0;       // this lane's row and first column (image coordinates)
    int W, H;
    int64_t pix0;        // packed index of (row, col0)
};

// Decodes item = tile << 3 | split << 2 | part into this lane's pixels. A whole tile (PX = 4)
// is 16 rows of 4 lanes with 4 adjacent pixels each; a split tile's part is 16 / (4 PX)
// of its rows: halves (PX = 2, 8 rows of 8 lanes) or quarters (PX = 1, 4 rows of 16 lanes).
template <int PX>
__device__ inline ItemPixels item_pixels(const gs_camera *__restrict__ cams, int n_cams,
                                         const int32_t *__restrict__ ranges, int item, int lane)
{
    constexpr int kLanesPerRow = kTile / PX;
    ItemPixels t;
    const int tile = item >> kItemTileShift, part = PX == 4 ? 0 : (item & 3);
    const int c = camera_of_tile(cams, n_cams, tile);
    const int local = tile - cams[c].tile_offset;
    const int tx_n = cams[c].tiles_x;
    const int ty = local / tx_n, tx = local - ty * tx_n;
    t.W = cams[c].width;
    t.H = cams[c].height;
    t.row = ty * kTile + part * (kWave / kLanesPerRow) + lane / kLanesPerRow;
    t.col0 = tx * kTile + (lane % kLanesPerRow) * PX;
    t.pix0 = cams[c].pixel_offset + (int64_t)t.row * t.W + t.col0;
    t.start = ranges[2 * tile];
    t.end = ranges[2 * tile + 1];
    return t;
}

// alpha_raw for one pixel given the lane's shared row terms; identical in forward and backward.
__device__ __forceinline__ float alpha_raw(const RasterRec &r, double dx, double bdy, double cdl)
{
    const double e = __builtin_fma(__builtin_fma(r.A, dx, bdy), dx, cdl);
    return __builtin_amdgcn_exp2f((float)e);
}

// Records of a batch that cannot reach alpha_min at any pixel the walk still changes are
// skipped by both walks: for them every such pixel's alpha is below alpha_min, so their step
// is a no-op (T, the colour, the last index and every gradient sum stay unchanged). The test
// is made once per record and batch, by the lane that gathered it, against the rectangle of
// the pixel centres of the lanes still active: with an unfinished pixel in the forward, with a
// pixel whose last entry is at or after the batch's first in the backward (a finished pixel,
// or one past its last entry, takes no step).
struct WaveRect {
    double x_lo, x_hi, y_lo, y_hi;   // pixel centres of the wave: [x_lo, x_hi] x [y_lo, y_hi]
    double thr;                       // log2(alpha_min) less a margin
};

template <int PX>
__device__ inline WaveRect wave_rect(const ItemPixels &t, const gs_params &prm)
{
    // lane 0 holds the first row and column, lane 63 the last row and the last lane's columns
    WaveRect w;
    w.x_lo = (double)__builtin_amdgcn_readlane(t.col0, 0) + 0.5;
    w.x_hi = (double)__builtin_amdgcn_readlane(t.col0, kWave - 1) + (double)(PX - 1) + 0.5;
    w.y_lo = (double)__builtin_amdgcn_readlane(t.row, 0) + 0.5;
    w.y_hi = (double)__builtin_amdgcn_readlane(t.row, kWave - 1) + 0.5;
    // the margin (2^-10) is far above the rounding of the per-pixel exponent, its float32
    // conversion and exp2; with alpha_min <= 0 the threshold is -inf or NaN and nothing is skipped
    w.thr = log2((double)prm.alpha_min) - 0x1p-10;
    return w;
}

// The rectangle of the pixel centres of the lanes in `act` (a lane mask, not empty) within
// the wave's rectangle `w`: lanes are laid out row-major, 16 / PX lanes per pixel row, each
// with PX adjacent pixels. Scalar arithmetic on the mask only.
template <int PX>
__device__ inline WaveRect lanes_rect(const WaveRect &w, uint64_t act)
{
    constexpr int kLanesPerRow = kTile / PX;
    uint64_t cols = act;   // fold the rows onto the first: bit c set when column c has an active lane
#pragma unroll
    for (int sh = 32; sh >= kLanesPerRow; sh >>= 1) cols |= cols >> sh;
    cols &= (1ull << kLanesPerRow) - 1;
    const int c_lo = (int)__builtin_ctzll(cols), c_hi = 63 - (int)__builtin_clzll(cols);
    const int l_lo = (int)__builtin_ctzll(act), l_hi = 63 - (int)__builtin_clzll(act);
    WaveRect r = w;
    r.x_lo = w.x_lo + (double)(c_lo * PX);
    r.x_hi = w.x_lo + (double)(c_hi * PX + PX - 1);
    r.y_lo = w.y_lo + (double)(l_lo / kLanesPerRow);
    r.y_hi = w.y_lo + (double)(l_hi / kLanesPerRow);
    return r;
}

// True when the gathered record cannot reach alpha_min inside the rectangle (the pixel
// centres of the lanes that are still active, lanes_rect). The exponent
// lo + A dx^2 + B dx dy + C dy^2 (a concave quadratic) is at least thr only inside an ellipse
// around mu' whose bounding box has half-widths sqrt(k (-4C) / D) and sqrt(k (-4A) / D), with
// k = lo - thr and D = 4AC - B^2. The record is skipped when k < 0, when that box, widened by
// a relative 2^-20 and an absolute 2^-20, misses the rectangle, or when the largest exponent
// over the rectangle is below thr: with mu' outside the rectangle that largest value lies on
// an edge that faces mu', and on an edge the quadratic is a concave parabola whose largest
// value is at its vertex clamped to the edge (the ellipse of a thin, tilted splat can miss a
// rectangle its bounding box meets). The D test bounds the relative rounding of those values by about
// 2^-32, and they are compared with a relative allowance of 2^-28. Records whose D carries
// more than 2^-20 relative cancellation, and any NaN, are kept.
// A float64 field of the gathered record from its two 32-bit halves (low word first).
__device__ __forceinline__ double rec_f64(float lo_word, float hi_word)
{
    return __hiloint2double(__float_as_int(hi_word), __float_as_int(lo_word));
}

__device__ inline bool record_misses(const Gathered &g, const WaveRect &w)
{
    // the fields are taken from the registers directly (RasterRec layout: mx, my, lo in q0;
    // A, B in q1; C in q2), so no copy of the record is made in memory
    const double lo = rec_f64(g.q0.z, g.q0.w), A = rec_f64(g.q1.x, g.q1.y), B = rec_f64(g.q1.z, g.q1.w),
                 C = rec_f64(g.q2.x, g.q2.y);
    const double k = lo - w.thr;
    if (k < 0.0) return true;
    const double ac4 = 4.0 * A * C, bb = B * B, D = ac4 - bb;
    if (!(D * 0x1p20 > ac4 + bb)) return false;
    const double sx = sqrt(k * (-4.0 * C) / D) * (1.0 + 0x1p-20) + 0x1p-20;
    const double sy = sqrt(k * (-4.0 * A) / D) * (1.0 + 0x1p-20) + 0x1p-20;
    const double mx = g.q0.x, my = g.q0.y;
    if (mx + sx < w.x_lo || mx - sx > w.x_hi || my + sy < w.y_lo || my - sy > w.y_hi) return true;
    if (!(A < 0.0) || (mx >= w.x_lo && mx <= w.x_hi && my >= w.y_lo && my <= w.y_hi)) return false;
    // only the edges that face mu' can hold the largest value (for a positive definite form
    // the constrained maximum never lies inside an edge whose outward side points away from mu')
    const double dx0 = w.x_lo - mx, dx1 = w.x_hi - mx, dy0 = w.y_lo - my, dy1 = w.y_hi - my;
    auto quad = [&](double dx, double dy) { return __builtin_fma(__builtin_fma(A, dx, B * dy), dx, C * dy * dy); };
    double best = -INFINITY;
    if (dx0 > 0.0 || dx1 < 0.0) {   // the edge x = x_lo or x = x_hi; its vertex at dy = B dx / (-2C)
        const double dx = dx0 > 0.0 ? dx0 : dx1;
        best = quad(dx, fmin(fmax(B * dx * (-0.5 / C), dy0), dy1));
    }
    if (dy0 > 0.0 || dy1 < 0.0) {   // the edge y = y_lo or y = y_hi; its vertex at dx = B dy / (-2A)
        const double dy = dy0 > 0.0 ? dy0 : dy1;
        best = fmax(best, quad(fmin(fmax(B * dy * (-0.5 / A), dx0), dx1), dy));
    }
    return best * (1.0 - 0x1p-28) < -k;
}

// Work-list cursor of a wave: positions [pos, end) taken from the counter and not yet used.
struct ItemCursor {
    int pos, end;
};

// First positions of a wave: wave w of the grid takes positions [w grab, (w + 1) grab)
// without an atomic. Every wave starts at once, and one same-address atomic per wave would
// serialise the start of the launch (about 34 ns each on this GPU: 140 us for 4096 waves).
__device__ inline ItemCursor first_cursor(int grab)
{
    const int w = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kBlockWaves + (int)(threadIdx.x >> 6));
    return ItemCursor{w * grab, (w + 1) * grab};
}

// Next item for this wave, or -1. After the first positions (first_cursor), the counter hands
// out the positions that follow them, `grab` consecutive ones per atomic (one address serves
// every wave, so fewer atomics help when items are many and short); the last wave to find the
// list exhausted resets the counters.
__device__ inline int next_item(int32_t *__restrict__ sched, int counter, int n_items, int grab, ItemCursor &cur,
                                int lane, int walk_stamp = 0)
{
    if (cur.pos >= cur.end) {
        int p = 0;
        if (lane == 0) p = atomicAdd(&sched[counter], grab) + (int)gridDim.x * kBlockWaves * grab;
        cur.pos = __builtin_amdgcn_readfirstlane(p);
        cur.end = cur.pos + grab;
    }
    const int pos = cur.pos++;
    if (pos < n_items) return __builtin_amdgcn_readfirstlane(sched[kSchedHeader + pos]);
    if (lane == 0) {
        const int waves = (int)gridDim.x * kBlockWaves;
        if (atomicAdd(&sched[counter + 1], 1) == waves - 1) {
            sched[counter] = 0;
            sched[counter + 1] = 0;
            if (walk_stamp) sched[kSchedWalkStamp] = walk_stamp;   // every item recorded its walk
        }
    }
    return -1;
}

// Issue priority of an unsplit tile (prio_len > 0): 2 when its walk has at least 2 prio_len
// entries, 1 from prio_len, else 0 (the walk: the list length, or the walk length the last
// rasterization recorded when it is shorter). Long walks are the end of the launch; under a
// full GPU a wave gets about a quarter of its SIMD, so the longest walks, started first,
// would run four times longer than alone. Graded levels give the longest the first claim on
// issue and let shorter ones fill the cycles they leave (split items take level 3).
__device__ inline int walk_priority(const int32_t *__restrict__ ranges, const int32_t *__restrict__ sched,
                                    int n_tiles, int item, int prio_len)
{
    if (prio_len <= 0) return 0;
    const int tile = item >> kItemTileShift;
    int len = ranges[2 * tile + 1] - ranges[2 * tile];
    if (sched[kSchedWalkStamp] == n_tiles) {
        const int walk = sched[sched_walk_offset(n_tiles) + tile];
        if (walk >= 1 && walk < len) len = walk;
    }
    return len >= 2 * prio_len ? 2 : len >= prio_len ? 1 : 0;
}

// s_setprio takes an immediate: one branch per level (wave-uniform)
__device__ inline void set_priority(int level)
{
    if (level >= 3) __builtin_amdgcn_s_setprio(3);
    else if (level == 2) __builtin_amdgcn_s_setprio(2);
    else if (level == 1) __builtin_amdgcn_s_setprio(1);
}

// ----------------------------------------------------------------------------- forward

// Per-pixel state of a work item. It is kept arithmetic so that every select depends on a
// single compare and no lane masks need combining: a skipped splat gets alpha = 0 (a no-op
// update), and during the forward walk a finished pixel carries T < 0 with |T| its final
// transmittance.
template <int PX>
struct PixState {
    double pyd, px0;   // centre of the lane's row and of its first pixel; pixel q is at px0 + q
    float T[PX], c0[PX], c1[PX], c2[PX];
    int last[PX], vis[PX];
};

template <int PX>
__device__ inline bool pixel_inside(const ItemPixels &t, int q)
{
    return t.row < t.H && t.col0 + q < t.W;
}

template <int PX>
__device__ inline void init_state(const ItemPixels &t, PixState<PX> &ps)
{
    ps.pyd = (double)t.row + 0.5;
    ps.px0 = (double)t.col0 + 0.5;
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        ps.T[q] = pixel_inside<PX>(t, q) ? 1.f : -1.f;
        ps.c0[q] = ps.c1[q] = ps.c2[q] = 0.f;
        ps.last[q] = ps.vis[q] = 0;
    }
}

// State of the forward at one list position: T (>= 0) and the colour so far.
template <int PX>
struct Snapshot {
    float T[PX], c0[PX], c1[PX], c2[PX];
};

template <int PX>
__device__ inline void take_snapshot(const PixState<PX> &ps, Snapshot<PX> &sn)
{
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        sn.T[q] = fabsf(ps.T[q]);
        sn.c0[q] = ps.c0[q];
        sn.c1[q] = ps.c1[q];
        sn.c2[q] = ps.c2[q];
    }
}

// Front-to-back walk of the item's list (eq. 7). On return T holds |T_final|. With
// snap_pos set (a list position t.start + 64 m), sn receives the state before entry
// snap_pos (the final state if the walk ends earlier). Returns the number of list entries
// the walk went through (to the batch in which its last pixel finished).
template <int PX, bool kVisited, int B>
__device__ inline int fwd_walk(const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids, const ItemPixels &t,
                                const gs_params &prm, PixState<PX> &ps, int snap_pos = -1,
                                Snapshot<PX> *sn = nullptr)
{
    bool snapped = snap_pos < 0;
    int walked = t.end - t.start;
    int stepped = 0;   // list slots walked (work counters)
    const WaveRect wr = wave_rect<PX>(t, prm);
    RasterRec *slice = wave_slice();
    const int lane = threadIdx.x & (kWave - 1);
    // batch k covers entries [t.start + 64 k, ...): its slots are loaded two batches ahead,
    // its records one batch ahead
    Gathered next = gather(rr, load_ids(ids, t.start, min(B, t.end - t.start), lane));
    int nid = load_ids(ids, t.start + B, min(B, t.end - t.start - B), lane);
    for (int b = t.start; b < t.end; b += B) {
        if (!snapped && b == snap_pos) {
            take_snapshot<PX>(ps, *sn);
            snapped = true;
        }
        const int nb = min(B, t.end - b);
        float tmax = ps.T[0];
#pragma unroll
        for (int q = 1; q < PX; ++q) tmax = fmaxf(tmax, ps.T[q]);
        const uint64_t act = __ballot(tmax >= 0.f);     // lanes with an unfinished pixel
        if (act == 0) {                                  // every pixel of the item is finished
            walked = b - t.start;
            break;
        }
        // records that miss the unfinished pixels are left out of the staged batch; the
        // counting pass (kVisited) counts every pair it reaches and keeps them all
        const WaveRect ar = lanes_rect<PX>(wr, act);
        const uint64_t keep = __ballot(lane < nb && (kVisited || !record_misses(next, ar)));
        const int np = stage_packed(slice, next, keep, lane, b - t.start + lane + 1);
        if (b + B < t.end) next = gather(rr, nid);
        if (b + 2 * B < t.end) nid = load_ids(ids, b + 2 * B, min(B, t.end - b - 2 * B), lane);
        // whole groups of staged slots, straight-line code inside a group (constant LDS
        // offsets, no per-entry branch), with the all-finished test between groups
        RasterRec rn = slice[0];
        for (int j0 = 0; j0 < np; j0 += kGroup) {
            if (j0 > 0) {
                float m = ps.T[0];
#pragma unroll
                for (int q = 1; q < PX; ++q) m = fmaxf(m, ps.T[q]);
                if (__ballot(m >= 0.f) == 0) break;
            }
            stepped += kGroup;
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
            // the next record is read while this one is composited, and no further: the
            // barrier lets only VALU and SALU work move across it, so later LDS reads are not
            // hoisted (two records in registers at most)
            const RasterRec r = rn;
            rn = slice[j < kGroup - 1 ? j0 + j + 1 : min(j0 + kGroup, B - 1)];
            __builtin_amdgcn_sched_barrier(0x0006);
            const double dy = (double)r.my - ps.pyd;
            const double bdy = r.B * dy;
            const double cdl = __builtin_fma(r.C * dy, dy, r.lo);
            const double dx0 = (double)r.mx - ps.px0;
            const int pos1 = staged_p1(r);
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                const double dx = dx0 - (double)q;   // exact: both sides are small binary fractions
                float a = __builtin_amdgcn_fmed3f(alpha_raw(r, dx, bdy, cdl), 0.f, prm.alpha_max);
                a = a < prm.alpha_min ? 0.f : a;                 // skipped: a no-op update
                if (kVisited) ps.vis[q] += (ps.T[q] >= 0.f && pos1 > 0) ? 1 : 0;   // padding not counted
                // T (1 - alpha) as T - T alpha with one rounding: the termination test sees T
                // with one rounding per factor (besides the error of alpha itself)
                const float Tn = __builtin_fmaf(-ps.T[q], a, ps.T[q]);
                const bool stop = Tn < prm.T_min;                // also true once finished (T < 0)
                const float w = stop ? 0.f : a * ps.T[q];
                ps.c0[q] = __builtin_fmaf(r.c0, w, ps.c0[q]);
                ps.c1[q] = __builtin_fmaf(r.c1, w, ps.c1[q]);
                ps.c2[q] = __builtin_fmaf(r.c2, w, ps.c2[q]);
                ps.last[q] = w > 0.f ? pos1 : ps.last[q];
                ps.T[q] = stop ? -fabsf(ps.T[q]) : Tn;
            }
            }
        }
    }
    if (!snapped) take_snapshot<PX>(ps, *sn);
#pragma unroll
    for (int q = 0; q < PX; ++q) ps.T[q] = fabsf(ps.T[q]);
    if (g_work_count && lane == 0) atomicAdd(&g_work_count[0], (unsigned long long)stepped * (kWave * PX));
    return walked;
}

// Records the forward walk length of the item's tile for the next work list (whole tiles,
// and part 0 of a split tile).
__device__ inline void record_walk(int32_t *__restrict__ sched, int n_tiles, int item, int walked)
{
    if ((item & 0x1B) == 0 && (threadIdx.x & (kWave - 1)) == 0)   // seg 0 and part 0
        sched[sched_walk_offset(n_tiles) + (item >> kItemTileShift)] = walked;
}

__device__ inline int wave_max(int v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v = max(v, __shfl_xor(v, d, kWave));
    return v;
}

struct BwdOut {
    int64_t n_splats, n_gauss;
    double *d_mean2d, *d_conic;
    float *d_colors, *d_opac;
    int atomic_lanes;   // up to this many contributing lanes, a splat's slot takes LDS atomics
};

// Per-wave gradient sums of the batch being walked: one slot per staged record, holding
//   sum v, sum v dx, sum v dy, sum v dx^2, sum v dx dy, sum v dy^2   (float64)
//   sum alpha T dL/dC(k), k = 0..2                                 (float32)
// over the wave's pixels. After each splat the wave fills that splat's slot in one of two
// ways, chosen by the number of lanes with a composited pixel (wave-uniform):
//   few lanes, at most the tuning's atomic_lanes (small splats, the common case at 1M
//     Gaussians): those lanes add their terms into the slot with LDS atomics, which
//     conflict only among themselves;
//   many lanes (large splats): a DPP reduction over the wave, and lane 63 writes the
//     totals into the slot (the splat's only writer).
// When the batch is done, lane j moves slot j to global memory with one atomic per term,
// so the global atomics of a batch are 9 instructions with up to 64 distinct addresses.
struct WaveAcc {
    double d[6][kBatch];
    float f[3][kBatch];
};

__device__ inline WaveAcc *wave_acc()
{
    __shared__ WaveAcc acc[kBlockWaves];
    return &acc[__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))];
}

__device__ inline void acc_clear(WaveAcc *acc, int lane)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) acc->d[k][lane] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) acc->f[k][lane] = 0.f;
}

__device__ inline void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Lane j < nk (the staged records) moves slot j (the splat of staged record j) to the global
// gradients and clears it:
//   dL/dmu' = -Y sum v Delta, with Y = -(2A, B; B, 2C) / log2(e)
//   dL/dY = -1/2 sum v Delta Delta^T,  dL/dc(k) = sum alpha T dL/dC(k),  dL/do = sum v / o
// The staged copy carries the list position in place of o, so 1/o is recovered as
// exp2(-lo) in float32 (lo = log2(o)): a splat reaches this point only with o >= alpha_min,
// so |lo| <= 8 for alpha_min = 1/255 and the relative error of 1/o is below 1e-6.
__device__ inline void acc_flush(const RasterRec *slice, WaveAcc *acc, int nk, int lane, const BwdOut &out)
{
    // LDS operations of one wave complete in order, so the slot reads below see every add
    __builtin_amdgcn_wave_barrier();
    if (lane < nk) {
        const double s_v = acc->d[0][lane], s_x = acc->d[1][lane], s_y = acc->d[2][lane];
        const double s_xx = acc->d[3][lane], s_xy = acc->d[4][lane], s_yy = acc->d[5][lane];
        const float s_c0 = acc->f[0][lane], s_c1 = acc->f[1][lane], s_c2 = acc->f[2][lane];
        if (s_v != 0.0 || s_xx != 0.0 || s_c0 != 0.f || s_c1 != 0.f || s_c2 != 0.f) {
            const RasterRec r = slice[lane];
            const int id = r.slot;
            const double il = 1.0 / kLog2eD;
            atomic_add_f64(&out.d_mean2d[id], (2.0 * r.A * s_x + r.B * s_y) * il);
            atomic_add_f64(&out.d_mean2d[out.n_splats + id], (r.B * s_x + 2.0 * r.C * s_y) * il);
            atomic_add_f64(&out.d_conic[id], -0.5 * s_xx);
            atomic_add_f64(&out.d_conic[out.n_splats + id], -0.5 * s_xy);
            atomic_add_f64(&out.d_conic[2 * out.n_splats + id], -0.5 * s_yy);
            atomic_add_f32(&out.d_colors[r.src], s_c0);
            atomic_add_f32(&out.d_colors[out.n_gauss + r.src], s_c1);
            atomic_add_f32(&out.d_colors[2 * out.n_gauss + r.src], s_c2);
            atomic_add_f32(&out.d_opac[r.src], (float)(s_v * (double)__builtin_amdgcn_exp2f(-(float)r.lo)));
        }
    }
    acc_clear(acc, lane);
    __builtin_amdgcn_wave_barrier();
}

// Back-to-front walk (Sec. 3.1) over the list positions [lo, hi) (the whole list: lo =
// t.start, hi = t.end). On entry T holds each pixel's transmittance after entry hi - 1
// (T_final for the whole list), gS the sum of dL/dC(k) S(k) over the entries from hi on
// (zero for the whole list), last the start positions and g0..g2 the upstream gradient
// dL/dC of each pixel.
template <int PX, int B>
__device__ inline void bwd_walk(const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids, const ItemPixels &t,
                                const gs_params &prm, const PixState<PX> &ps, float (&T)[PX], float (&gS)[PX],
                                const float (&g0)[PX], const float (&g1)[PX], const float (&g2)[PX],
                                const BwdOut &out, int lo, int hi)
{
    const int lane = threadIdx.x & (kWave - 1);
    int maxlast = 0;
#pragma unroll
    for (int q = 0; q < PX; ++q) maxlast = max(maxlast, ps.last[q]);
    maxlast = __builtin_amdgcn_readfirstlane(wave_max(maxlast));
    const int kend = min(hi, t.start + maxlast);
    if (kend <= lo) return;
    const WaveRect wr = wave_rect<PX>(t, prm);
    RasterRec *slice = wave_slice();
    WaveAcc *acc = wave_acc();
    acc_clear(acc, lane);
    int stepped = 0;   // list slots walked (work counters)
    // batches run back to front: [bstart, bend) with bend = kend, kend - 64, ...
    // batch k covers entries [max(lo, e_k - 64), e_k) with e_k = kend - 64 k: its slots
    // are loaded two batches ahead, its records one batch ahead
    const int s0 = max(lo, kend - B);
    Gathered next = gather(rr, load_ids(ids, s0, kend - s0, lane));
    int nid = -1;
    if (s0 > lo) {
        const int s1 = max(lo, s0 - B);
        nid = load_ids(ids, s1, s0 - s1, lane);
    }
    int lane_last = 0;   // the lane's pixels are active for list positions up to this one
#pragma unroll
    for (int q = 0; q < PX; ++q) lane_last = max(lane_last, ps.last[q]);
    for (int bend = kend; bend > lo; bend -= B) {
        const int bstart = max(lo, bend - B);
        const int nb = bend - bstart;
        // records that miss the pixels active in this batch (last at or after its first
        // entry) are left out of the staged batch; some lane is active, since kend is the
        // largest last
        const uint64_t act = __ballot(lane_last >= bstart - t.start + 1);
        const WaveRect ar = lanes_rect<PX>(wr, act);
        const uint64_t keep = __ballot(lane < nb && !record_misses(next, ar));
        const int nk = __popcll(keep);
        stepped += nk;
        stage_packed(slice, next, keep, lane, bstart - t.start + lane + 1);
        if (bstart > lo) next = gather(rr, nid);
        const int e2 = bstart - B;   // end of the batch after next
        if (e2 > lo) {
            const int s2 = max(lo, e2 - B);
            nid = load_ids(ids, s2, e2 - s2, lane);
        }
        RasterRec rn = slice[max(nk - 1, 0)];
        for (int j = nk - 1; j >= 0; --j) {
            // the next record (j - 1) is read while this one is processed
            const RasterRec r = rn;
            rn = slice[max(j - 1, 0)];
            const int pos1 = staged_p1(r);
            const double dy = (double)r.my - ps.pyd;
            const double dx0 = (double)r.mx - ps.px0;
            const double bdy = r.B * dy;
            const double cdl = __builtin_fma(r.C * dy, dy, r.lo);
            // per-lane sums over the lane's pixels; the lane's pixels share one row, so the
            // dy-weighted sums follow from sum v and sum v dx. The position sums are float64:
            // dL/dY along the thin axis of a needle-like splat is a small difference of
            // these sums, which float32 rounding would swamp. (Float32 moments sum q^k v of
            // the lane's pixels, combined in float64 once per splat, lost enough of it to move
            // single quaternion gradients past the 1e-3 bar.)
            double s_v = 0.0, s_x = 0.0, s_xx = 0.0;
            float s_c0 = 0.f, s_c1 = 0.f, s_c2 = 0.f;
            float live_sum = 0.f;
#pragma unroll
            for (int q = 0; q < PX; ++q) {
                // inactive (past `last`) or skipped pairs get alpha = 0: then rcp(1 - alpha) = 1,
                // w = 0 and v = 0, and the pair changes nothing
                const double dx = dx0 - (double)q;
                const float a_raw = alpha_raw(r, dx, bdy, cdl);
                float a = __builtin_amdgcn_fmed3f(a_raw, 0.f, prm.alpha_max);
                a = pos1 <= ps.last[q] ? a : 0.f;
                a = a < prm.alpha_min ? 0.f : a;
                live_sum += a;
                const float rinv = __builtin_amdgcn_rcpf(1.f - a);
                T[q] *= rinv;                                      // T before this splat (eq. 17)
                const float w = a * T[q];
                s_c0 = __builtin_fmaf(w, g0[q], s_c0);               // eq. (16)
                s_c1 = __builtin_fmaf(w, g1[q], s_c1);
                s_c2 = __builtin_fmaf(w, g2[q], s_c2);
                const float gc = g0[q] * r.c0 + g1[q] * r.c1 + g2[q] * r.c2;
                const float dalpha = gc * T[q] - gS[q] * rinv;      // eq. (18)
                gS[q] = __builtin_fmaf(gc, w, gS[q]);
                // eq. (19): dalpha/dsigma = -alpha; a clamped alpha passes no gradient to o or sigma
                const double v = (double)(a_raw > prm.alpha_max ? 0.f : dalpha * a);
                const double vx = v * dx;
                s_v += v;
                s_x += vx;
                s_xx = __builtin_fma(vx, dx, s_xx);
            }
            const uint64_t live = __ballot(live_sum > 0.f);
            if (live == 0) continue;
            if (__popcll(live) <= out.atomic_lanes) {
                const double s_y = s_v * dy, s_xy = s_x * dy;
                const double s_yy = s_y * dy;
                if (live_sum > 0.f) {
                    lds_add(&acc->d[0][j], s_v);
                    lds_add(&acc->d[1][j], s_x);
                    lds_add(&acc->d[2][j], s_y);
                    lds_add(&acc->d[3][j], s_xx);
                    lds_add(&acc->d[4][j], s_xy);
                    lds_add(&acc->d[5][j], s_yy);
                    lds_add(&acc->f[0][j], s_c0);
                    lds_add(&acc->f[1][j], s_c1);
                    lds_add(&acc->f[2][j], s_c2);
                }
            } else {
                // reduce over the wave: first over the lanes of one pixel row (they share
                // dy, so the dy-weighted sums follow from the row's sums), then within rows
                // of 16 lanes and across rows; lane 63 writes the totals: the slot has no
                // other writer for this splat
                constexpr int kRowLevels = PX == 4 ? 2 : PX == 2 ? 3 : 4;   // log2 lanes per pixel row
                s_v = row_levels<0, kRowLevels>(s_v);
                s_x = row_levels<0, kRowLevels>(s_x);
                s_xx = row_levels<0, kRowLevels>(s_xx);
                double s_y = s_v * dy, s_xy = s_x * dy;
                double s_yy = s_y * dy;
                s_v = rows_to_lane63(row_levels<kRowLevels, 4>(s_v));
                s_x = rows_to_lane63(row_levels<kRowLevels, 4>(s_x));
                s_y = rows_to_lane63(row_levels<kRowLevels, 4>(s_y));
                s_xx = rows_to_lane63(row_levels<kRowLevels, 4>(s_xx));
                s_xy = rows_to_lane63(row_levels<kRowLevels, 4>(s_xy));
                s_yy = rows_to_lane63(row_levels<kRowLevels, 4>(s_yy));
                s_c0 = rows_to_lane63(row_sum(s_c0));
                s_c1 = rows_to_lane63(row_sum(s_c1));
                s_c2 = rows_to_lane63(row_sum(s_c2));
                if (lane == kWave - 1) {
                    acc->d[0][j] = s_v;
                    acc->d[1][j] = s_x;
                    acc->d[2][j] = s_y;
                    acc->d[3][j] = s_xx;
                    acc->d[4][j] = s_xy;
                    acc->d[5][j] = s_yy;
                    acc->f[0][j] = s_c0;
                    acc->f[1][j] = s_c1;
                    acc->f[2][j] = s_c2;
                }
            }
        }
        acc_flush(slice, acc, nk, lane, out);
    }
    if (g_work_count && lane == 0) atomicAdd(&g_work_count[1], (unsigned long long)stepped * (kWave * PX));
}

// ----------------------------------------------------------------------------- kernels

struct FwdOut {
    int64_t n_pixels;
    float *image, *T_out;
    int32_t *last_out, *visited_out;
};

template <int PX, bool kVisited, int B>
__device__ inline void fwd_item(const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids,
                                const ItemPixels &t, const gs_params &prm, const FwdOut &o, int32_t *sched,
                                int n_tiles, int item)
{
    PixState<PX> ps;
    init_state<PX>(t, ps);
    record_walk(sched, n_tiles, item, fwd_walk<PX, kVisited, B>(rr, ids, t, prm, ps));
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        if (pixel_inside<PX>(t, q)) {
            const int64_t pix = t.pix0 + q;
            // the background is seen through T_final (exactly C when it is zero)
            o.image[pix] = __builtin_fmaf(ps.T[q], prm.background[0], ps.c0[q]);
            o.image[o.n_pixels + pix] = __builtin_fmaf(ps.T[q], prm.background[1], ps.c1[q]);
            o.image[2 * o.n_pixels + pix] = __builtin_fmaf(ps.T[q], prm.background[2], ps.c2[q]);
            o.T_out[pix] = ps.T[q];
            o.last_out[pix] = ps.last[q];
            if (kVisited) o.visited_out[pix] = ps.vis[q];
        }
    }
}

template <bool kVisited, int B>
__global__ __launch_bounds__(kWave * kBlockWaves) void raster_fwd_kernel(
    const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids, const int32_t *__restrict__ ranges,
    int32_t *__restrict__ sched, const gs_camera *__restrict__ cams, int n_cams, gs_params prm, FwdOut o, int prio, int grab, int prio_len,
    int n_tiles)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int n_items = __builtin_amdgcn_readfirstlane(sched[kSchedItems]);
    const int parts = __builtin_amdgcn_readfirstlane(sched[kSchedParts]);
    ItemCursor cur = first_cursor(grab);
    for (;;) {
        const int item = next_item(sched, kSchedFwd, n_items, grab, cur, lane, n_tiles);
        if (item < 0) break;
        if ((item >> 3) & 3) continue;   // a backward segment of the fused kernel
        if (item & 4) {
            if (prio) set_priority(3);
            if (parts == 4)
                fwd_item<1, kVisited, B>(rr, ids, item_pixels<1>(cams, n_cams, ranges, item, lane), prm, o, sched, n_tiles,
                                      item);
            else
                fwd_item<2, kVisited, B>(rr, ids, item_pixels<2>(cams, n_cams, ranges, item, lane), prm, o, sched, n_tiles,
                                      item);
            __builtin_amdgcn_s_setprio(0);
        } else {
            set_priority(__builtin_amdgcn_readfirstlane(walk_priority(ranges, sched, n_tiles, item, prio_len)));
            fwd_item<4, kVisited, B>(rr, ids, item_pixels<4>(cams, n_cams, ranges, item, lane), prm, o, sched, n_tiles,
                                  item);
            __builtin_amdgcn_s_setprio(0);
        }
    }
}

struct BwdIn {
    int64_t n_pixels;
    const float *dL_dimage, *T_final;
    const int32_t *last_in;
};

template <int PX, int B>
__device__ inline void bwd_item(const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids,
                                const ItemPixels &t, const gs_params &prm, const BwdIn &in, const BwdOut &out)
{
    PixState<PX> ps;
    init_state<PX>(t, ps);
    float T[PX], g0[PX], g1[PX], g2[PX];
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        T[q] = 1.f;
        g0[q] = g1[q] = g2[q] = 0.f;
        if (pixel_inside<PX>(t, q)) {
            const int64_t pix = t.pix0 + q;
            T[q] = in.T_final[pix];
            ps.last[q] = in.last_in[pix];
            g0[q] = in.dL_dimage[pix];
            g1[q] = in.dL_dimage[in.n_pixels + pix];
            g2[q] = in.dL_dimage[2 * in.n_pixels + pix];
        }
    }
    // the background is the colour behind the last entry, seen with weight T_final
    float gS[PX];
#pragma unroll
    for (int q = 0; q < PX; ++q)
        gS[q] = (g0[q] * prm.background[0] + g1[q] * prm.background[1] + g2[q] * prm.background[2]) * T[q];
    bwd_walk<PX, B>(rr, ids, t, prm, ps, T, gS, g0, g1, g2, out, t.start, t.end);
}

template <int B>
__global__ __launch_bounds__(kWave * kBlockWaves) __attribute__((amdgpu_waves_per_eu(4))) void raster_bwd_kernel(
    const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids, const int32_t *__restrict__ ranges,
    int32_t *__restrict__ sched, const gs_camera *__restrict__ cams, int n_cams, gs_params prm, BwdIn in, BwdOut out,
    int prio, int grab, int prio_len, int n_tiles)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int n_items = __builtin_amdgcn_readfirstlane(sched[kSchedItems]);
    const int parts = __builtin_amdgcn_readfirstlane(sched[kSchedParts]);
    ItemCursor cur = first_cursor(grab);
    for (;;) {
        const int item = next_item(sched, kSchedBwd, n_items, grab, cur, lane);
        if (item < 0) break;
        if ((item >> 3) & 3) continue;   // a backward segment of the fused kernel
        if (item & 4) {
            if (prio) set_priority(3);
            if (parts == 4)
                bwd_item<1, B>(rr, ids, item_pixels<1>(cams, n_cams, ranges, item, lane), prm, in, out);
            else
                bwd_item<2, B>(rr, ids, item_pixels<2>(cams, n_cams, ranges, item, lane), prm, in, out);
            __builtin_amdgcn_s_setprio(0);
        } else {
            set_priority(__builtin_amdgcn_readfirstlane(walk_priority(ranges, sched, n_tiles, item, prio_len)));
            bwd_item<4, B>(rr, ids, item_pixels<4>(cams, n_cams, ranges, item, lane), prm, in, out);
            __builtin_amdgcn_s_setprio(0);
        }
    }
}

// Fused training step of one item: forward, dL/dC = 2 (C - target) in registers, backward.
struct FusedIO {
    int64_t n_pixels;
    const float *target;
    float *image;   // optional
    float *loss;    // optional, accumulated sum of (C - target)^2
    const int64_t *list_flags;   // gs_bins.counters: [1] != 0 when the list was not built
};

template <int PX, int B>
__device__ inline void fused_item(const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids,
                                  const ItemPixels &t, const gs_params &prm, const FusedIO &io, const BwdOut &out,
                                  int seg, int segs, int32_t *sched, int n_tiles, int item, float &loss_acc)
{
    // segment seg of segs: list positions [lo, hi), boundaries at multiples of 64 entries
    const int n = t.end - t.start;
    const int per = ((n + segs - 1) / segs + B - 1) / B * B;
    const int lo = min(t.end, t.start + seg * per);
    const int hi = seg == segs - 1 ? t.end : min(t.end, lo + per);
    PixState<PX> ps;
    init_state<PX>(t, ps);
    Snapshot<PX> sn;
    const int walked = hi < t.end ? fwd_walk<PX, false, B>(rr, ids, t, prm, ps, hi, &sn)
                                  : fwd_walk<PX, false, B>(rr, ids, t, prm, ps);
    record_walk(sched, n_tiles, item, walked);
    float g0[PX], g1[PX], g2[PX];
    float l2 = 0.f;
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        g0[q] = g1[q] = g2[q] = 0.f;
        if (pixel_inside<PX>(t, q)) {
            const int64_t pix = t.pix0 + q;
            const float C0 = __builtin_fmaf(ps.T[q], prm.background[0], ps.c0[q]);
            const float C1 = __builtin_fmaf(ps.T[q], prm.background[1], ps.c1[q]);
            const float C2 = __builtin_fmaf(ps.T[q], prm.background[2], ps.c2[q]);
            const float d0 = C0 - io.target[pix];
            const float d1 = C1 - io.target[io.n_pixels + pix];
            const float d2 = C2 - io.target[2 * io.n_pixels + pix];
            g0[q] = 2.f * d0;
            g1[q] = 2.f * d1;
            g2[q] = 2.f * d2;
            l2 += d0 * d0 + d1 * d1 + d2 * d2;
            if (io.image && seg == 0) {
                io.image[pix] = C0;
                io.image[io.n_pixels + pix] = C1;
                io.image[2 * io.n_pixels + pix] = C2;
            }
        }
    }
    if (seg == 0) loss_acc += l2;   // summed over the wave's items, added to the loss once per wave
    // the walk back over [lo, hi) starts from the state after entry hi - 1: for the last
    // segment T_final and only the background behind (weight T_final); otherwise the
    // snapshot, with the colour added from hi on carried by gS = dL/dC . (C_final - C(hi))
    float T[PX], gS[PX];
#pragma unroll
    for (int q = 0; q < PX; ++q) {
        const float gbg = (g0[q] * prm.background[0] + g1[q] * prm.background[1] + g2[q] * prm.background[2]) * ps.T[q];
        if (hi < t.end) {
            T[q] = sn.T[q];
            gS[q] = g0[q] * (ps.c0[q] - sn.c0[q]) + g1[q] * (ps.c1[q] - sn.c1[q]) + g2[q] * (ps.c2[q] - sn.c2[q]) +
                    gbg;
        } else {
            T[q] = ps.T[q];
            gS[q] = gbg;
        }
    }
    bwd_walk<PX, B>(rr, ids, t, prm, ps, T, gS, g0, g1, g2, out, lo, hi);
}

template <int B>
__global__ __launch_bounds__(kWave * kBlockWaves) __attribute__((amdgpu_waves_per_eu(4))) void raster_fused_kernel(
    const RasterRec *__restrict__ rr, const int32_t *__restrict__ ids, const int32_t *__restrict__ ranges,
    int32_t *__restrict__ sched, const gs_camera *__restrict__ cams, int n_cams, gs_params prm, FusedIO io,
    BwdOut out, int prio, int grab, int prio_len, int n_tiles)
{
    const int lane = threadIdx.x & (kWave - 1);
    // no list (overflow or a failed sort): the step's result would be wrong, so the loss is
    // set to NaN, which the caller sees without a host synchronisation, and nothing is done
    if (io.list_flags[1] != 0) {
        if (io.loss && blockIdx.x == 0 && threadIdx.x == 0) *io.loss = __builtin_nanf("");
        return;
    }
    const int n_items = __builtin_amdgcn_readfirstlane(sched[kSchedItems]);
    const int parts = __builtin_amdgcn_readfirstlane(sched[kSchedParts]);
    const int segs = __builtin_amdgcn_readfirstlane(sched[kSchedSegs]);
    ItemCursor cur = first_cursor(grab);
    // this lane's share of the loss over the wave's items: one atomic per wave at the end, since
    // one per item queues on the loss's address once the items are short (the list's end)
    float loss_acc = 0.f;
    for (;;) {
        const int item = next_item(sched, kSchedFused, n_items, grab, cur, lane, n_tiles);
        if (item < 0) break;
        if (item & 4) {
            const int seg = (item >> 3) & 3;
            if (prio) set_priority(3);
            if (parts == 4)
                fused_item<1, B>(rr, ids, item_pixels<1>(cams, n_cams, ranges, item, lane), prm, io, out, seg, segs,
                              sched, n_tiles, item, loss_acc);
            else
                fused_item<2, B>(rr, ids, item_pixels<2>(cams, n_cams, ranges, item, lane), prm, io, out, seg, segs,
                              sched, n_tiles, item, loss_acc);
            __builtin_amdgcn_s_setprio(0);
        } else {
            set_priority(__builtin_amdgcn_readfirstlane(walk_priority(ranges, sched, n_tiles, item, prio_len)));
            fused_item<4, B>(rr, ids, item_pixels<4>(cams, n_cams, ranges, item, lane), prm, io, out, 0, 1, sched,
                          n_tiles, item, loss_acc);
            __builtin_amdgcn_s_setprio(0);
        }
    }
    if (io.loss) {
        const float l2 = wave_sum_to_lane63(loss_acc);
        if (lane == kWave - 1 && l2 != 0.f) atomic_add_f32(io.loss, l2);   // a NaN is added too
    }
}

static int check_raster_args(const gs_splats *s, const gs_bins *bins, const gs_camera *cams, int32_t n_cams,
                             const gs_params *prm, int64_t n_pixels)
{
    if (!s || !bins || !cams || !prm || n_cams < 1 || n_pixels < 0 || !s->raster || !bins->ids || !bins->ranges ||
        !bins->schedule || bins->n_tiles < 0)
        return set_error(GS_ERR_INVALID, "rasterize: null argument or bad size");
    if (!(prm->alpha_max > 0.0f && prm->alpha_max <= 1.0f))
        return set_error(GS_ERR_INVALID, "rasterize: alpha_max must be in (0, 1]");
    if (((uintptr_t)s->raster) & 63) return set_error(GS_ERR_INVALID, "rasterize: raster must be 64-byte aligned");
    return GS_OK;
}

// The thresholds as the kernels apply them. alpha_max = 1 (the literal image formation of
// eq. 7) becomes the largest float32 below 1: then 1 - alpha >= 2^-24 for every composited
// pair, so T after the pair stays positive and the backward's division of eq. (17) is
// defined. Only alphas within 6e-8 of 1 (opacities that close to 1) are affected.
static gs_params kernel_params(const gs_params *prm)
{
    gs_params k = *prm;
    if (k.alpha_max >= 1.0f) k.alpha_max = 0x1.fffffep-1f;
    return k;
}

}  // namespace gsx

using namespace gsx;

extern "C" int gs_set_work_counter(unsigned long long *counts)
{
    clear_error();
    return check_hip(hipMemcpyToSymbol(HIP_SYMBOL(g_work_count), &counts, sizeof(counts)), "gs_set_work_counter");
}

extern "C" int gs_rasterize_fwd(const gs_splats *s, const gs_bins *bins, const gs_camera *cams, int32_t n_cams,
                                const gs_params *prm, int64_t n_pixels, float *image, float *T_final,
                                int32_t *last, int32_t *visited, void *stream)
{
    clear_error();
    int rc = check_raster_args(s, bins, cams, n_cams, prm, n_pixels);
    if (rc != GS_OK) return rc;
    if (!image || !T_final || !last) return set_error(GS_ERR_INVALID, "gs_rasterize_fwd: null output");
    if (bins->n_tiles == 0) return GS_OK;
    // every tile is on the work list, empty ones included, so each pixel is written exactly once
    const dim3 grid(persistent_blocks(kBlockWaves)), block(kWave * kBlockWaves);
    const FwdOut o{n_pixels, image, T_final, last, visited};
    const gs_tuning &tu = current_tuning();
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, block, 0, (hipStream_t)stream, (const RasterRec *)s->raster, bins->ids,
                           bins->ranges, bins->schedule, cams, (int)n_cams, kernel_params(prm), o, tu.split_priority,
                           tu.item_grab, tu.prio_len, bins->n_tiles);
    };
    if (visited) {
        if (tu.batch == 32) launch(raster_fwd_kernel<true, 32>); else launch(raster_fwd_kernel<true, 64>);
    } else {
        if (tu.batch == 32) launch(raster_fwd_kernel<false, 32>); else launch(raster_fwd_kernel<false, 64>);
    }
    return check_launch("gs_rasterize_fwd");
}

static int check_bwd_outputs(const gs_splats *s, int64_t n_splats, const gs_params *prm, double *dL_dmean2d,
                             double *dL_dconic, int64_t n_gaussians, float *dL_dcolors, float *dL_dopac)
{
    if (!dL_dmean2d || !dL_dconic || !dL_dcolors || !dL_dopac || n_splats < 0 || n_splats > s->capacity ||
        n_gaussians < 1)
        return set_error(GS_ERR_INVALID, "rasterize backward: null gradient buffer or bad size");
    return GS_OK;
}

extern "C" int gs_rasterize_bwd(const gs_splats *s, int64_t n_splats, const gs_bins *bins, const gs_camera *cams,
                                int32_t n_cams, const gs_params *prm, int64_t n_pixels, const float *dL_dimage,
                                const float *T_final, const int32_t *last, double *dL_dmean2d, double *dL_dconic,
                                int64_t n_gaussians, float *dL_dcolors, float *dL_dopac, void *stream)
{
    clear_error();
    int rc = check_raster_args(s, bins, cams, n_cams, prm, n_pixels);
    if (rc != GS_OK) return rc;
    if (!dL_dimage || !T_final || !last) return set_error(GS_ERR_INVALID, "gs_rasterize_bwd: null input");
    rc = check_bwd_outputs(s, n_splats, prm, dL_dmean2d, dL_dconic, n_gaussians, dL_dcolors, dL_dopac);
    if (rc != GS_OK) return rc;
    if (bins->n_tiles == 0) return GS_OK;
    const BwdIn in{n_pixels, dL_dimage, T_final, last};
    const BwdOut out{n_splats, n_gaussians, dL_dmean2d, dL_dconic, dL_dcolors, dL_dopac,
                     current_tuning().atomic_lanes};
    const gs_tuning &tu = current_tuning();
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(persistent_blocks(kBlockWaves)), dim3(kWave * kBlockWaves), 0,
                           (hipStream_t)stream, (const RasterRec *)s->raster, bins->ids, bins->ranges, bins->schedule,
                           cams, (int)n_cams, kernel_params(prm), in, out, tu.split_priority, tu.item_grab, tu.prio_len,
                           bins->n_tiles);
    };
    if (tu.batch == 32) launch(raster_bwd_kernel<32>); else launch(raster_bwd_kernel<64>);
    return check_launch("gs_rasterize_bwd");
}

extern "C" int gs_rasterize_fused_l2(const gs_splats *s, int64_t n_splats, const gs_bins *bins,
                                     const gs_camera *cams, int32_t n_cams, const gs_params *prm, int64_t n_pixels,
                                     const float *target, float *image, float *loss, double *dL_dmean2d,
                                     double *dL_dconic, int64_t n_gaussians, float *dL_dcolors, float *dL_dopac,
                                     void *stream)
{
    clear_error();
    int rc = check_raster_args(s, bins, cams, n_cams, prm, n_pixels);
    if (rc != GS_OK) return rc;
    if (!target) return set_error(GS_ERR_INVALID, "gs_rasterize_fused_l2: null target");
    rc = check_bwd_outputs(s, n_splats, prm, dL_dmean2d, dL_dconic, n_gaussians, dL_dcolors, dL_dopac);
    if (rc != GS_OK) return rc;
    if (bins->n_tiles == 0) return GS_OK;
    if (!bins->counters) return set_error(GS_ERR_INVALID, "gs_rasterize_fused_l2: null bins->counters");
    const FusedIO io{n_pixels, target, image, loss, (const int64_t *)bins->counters};
    const BwdOut out{n_splats, n_gaussians, dL_dmean2d, dL_dconic, dL_dcolors, dL_dopac,
                     current_tuning().atomic_lanes};
    const gs_tuning &tu = current_tuning();
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(persistent_blocks(kBlockWaves)), dim3(kWave * kBlockWaves), 0,
                           (hipStream_t)stream, (const RasterRec *)s->raster, bins->ids, bins->ranges, bins->schedule,
                           cams, (int)n_cams, kernel_params(prm), io, out, tu.split_priority, tu.item_grab, tu.prio_len,
                           bins->n_tiles);
    };
    if (tu.batch == 32) launch(raster_fused_kernel<32>); else launch(raster_fused_kernel<64>);
    return check_launch("gs_rasterize_fused_l2");
}
