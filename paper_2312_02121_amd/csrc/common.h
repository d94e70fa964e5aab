// Internal helpers shared by the HIP translation units of libgsplat_mi355x.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsplat_mi355x.h"

namespace gsx {

constexpr int kTile = GS_TILE;           // tile edge in pixels
constexpr int kTilePixels = kTile * kTile;
constexpr int kWave = 64;                // CDNA wavefront width
constexpr int kRecFloats = 12;           // floats per splat record

// Compositing record of one splat (64 bytes, gs_splats.raster). The rasterizer gathers 64 of
// them per wave (one per lane, four 16-byte loads) into LDS and reads each back broadcast.
//   alpha_raw(dx, dy) = exp2(lo + A dx^2 + B dx dy + C dy^2),  (dx, dy) = mu' - pixel centre
// lo = log2(o); A = -log2(e)/2 Y00, B = -log2(e) Y01, C = -log2(e)/2 Y11 from the float32 conic.
// The quadratic form is evaluated in float64: for thin splats Y is nearly singular and the three
// terms cancel, which in float32 costs up to ~1e-5 of image accuracy. It is not free: measured
// on gfx950, a wave64 float64 FMA or add takes ~4.3 clocks of its SIMD against ~2.2 for a float32
// one, and a conversion ~3.4, so the per-pixel exponent (one subtraction, two FMAs and a
// conversion in float64) costs about as much as eight float32 operations.
struct alignas(64) RasterRec {
    float mx, my;     // mu', the same float32 values as in rec
    double lo;
    double A, B, C;
    float c0, c1, c2;
    float o;
    int src;          // scene Gaussian index
    int slot;         // the record's own splat slot (the gradient index of dL/dmu' and dL/dY)
};
static_assert(sizeof(RasterRec) == 64, "RasterRec must be 64 bytes");

constexpr double kLog2eD = 1.4426950408889634074;

// Rasterizer work list (gs_bins.schedule, int32). Header words, then the items.
// An item is tile << 5 | seg << 3 | split << 2 | part: split = 0 covers the whole tile,
// split = 1 one part of it (rows 16 / parts * part onward). A split tile has parts x segs
// items: seg is the item's segment of the tile's list in the fused kernel's backward (each
// such item runs the forward and walks back over its own segment); the forward and backward
// kernels take the seg 0 items only, over the whole list.
constexpr int kSchedItems = 0;      // number of items
constexpr int kSchedFwd = 1;        // forward kernel: next item, then finished-wave count
constexpr int kSchedBwd = 3;        // backward kernel: next item, then finished-wave count
constexpr int kSchedFused = 5;      // fused kernel: next item, then finished-wave count
constexpr int kSchedParts = 7;      // parts per split tile (2 or 4) the list was built with
constexpr int kSchedSegs = 40;      // backward list segments per split tile (1, 2 or 4)
constexpr int kSchedWalkStamp = 41; // n_tiles once the walk lengths below have been written
constexpr int kItemTileShift = 5;
constexpr int kMaxItemsPerTile = 16;   // parts x segs
constexpr int kSchedBuckets = 8;    // 16 bucket counts
constexpr int kSchedCursors = 24;   // 16 bucket cursors
constexpr int kSchedHeader = 64;
constexpr int kSchedNumBuckets = 16;
// After the items: int32 [n_tiles], the forward walk length of each tile (entries its
// forward evaluated) in the last rasterization with this work list. The next work list is
// built from min(list length, walk length) when the stamp matches: it orders and splits
// tiles by the work their walks did rather than by list length (tiles whose pixels saturate
// early have long lists and short walks). Only the schedule depends on it.
__host__ __device__ inline int64_t sched_walk_offset(int64_t n_tiles)
{
    return (int64_t)kSchedHeader + (int64_t)kMaxItemsPerTile * n_tiles;
}

// Workgroups for a persistent launch: enough waves to fill every SIMD of the device.
unsigned persistent_blocks(int waves_per_block);
int device_cu_count();   // compute units of the current device
const gs_tuning &current_tuning();

// ------------------------------------------------------------------ host-side status

int set_error(int code, const char *msg);   // records msg, returns code
int check_hip(hipError_t e, const char *what);
int check_launch(const char *what);         // hipGetLastError after a launch
void clear_error();

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// ------------------------------------------------------------------ device helpers

// Largest camera index c with cams[c].proj_offset <= p (cameras sorted by proj_offset).
__device__ inline int camera_of_splat(const gs_camera *__restrict__ cams, int n_cams, int64_t p)
{
    int lo = 0, hi = n_cams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cams[mid].proj_offset <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Largest camera index c with cams[c].tile_offset <= tile (cameras sorted by tile_offset).
__device__ inline int camera_of_tile(const gs_camera *__restrict__ cams, int n_cams, int tile)
{
    int lo = 0, hi = n_cams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cams[mid].tile_offset <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline uint64_t lanemask_lt()
{
    const unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Sum over the 64 lanes of a wave using DPP row operations; the total lands in lane 63.
__device__ inline float wave_sum_to_lane63(float v)
{
    // within rows of 16: xor-like butterflies via quad_perm, half-row and row mirrors
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false)); // quad_perm [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false)); // quad_perm [2,3,0,1]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false)); // row_half_mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false)); // row_mirror
    // across rows: lane 15 of each row into the next row, then lane 31 into rows 2 and 3
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false)); // row_bcast:15
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false)); // row_bcast:31
    return v;
}

// Sums within each row of 16 lanes (every lane of the row ends with its row's total),
// with butterflies whose DPP patterns write every lane, so no lane keeps an old value.
// float64 values move as two 32-bit halves.
template <int kCtrl>
__device__ inline double dpp_all_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), kCtrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Partial row sums: levels [kFrom, kTo) of the butterfly below (level 0: pairs, 1: quads,
// 2: half-rows of 8, 3: rows of 16 lanes).
template <int kFrom, int kTo>
__device__ inline double row_levels(double v)
{
    if constexpr (kFrom <= 0 && kTo > 0) v += dpp_all_f64<0xB1>(v);
    if constexpr (kFrom <= 1 && kTo > 1) v += dpp_all_f64<0x4E>(v);
    if constexpr (kFrom <= 2 && kTo > 2) v += dpp_all_f64<0x141>(v);
    if constexpr (kFrom <= 3 && kTo > 3) v += dpp_all_f64<0x140>(v);
    return v;
}

template <int kFrom, int kTo>
__device__ inline float row_levels(float v)
{
    if constexpr (kFrom <= 0 && kTo > 0)
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    if constexpr (kFrom <= 1 && kTo > 1)
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    if constexpr (kFrom <= 2 && kTo > 2)
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    if constexpr (kFrom <= 3 && kTo > 3)
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
    return v;
}

__device__ inline double row_sum(double v)
{
    v += dpp_all_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_all_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_all_f64<0x141>(v);   // row_half_mirror
    v += dpp_all_f64<0x140>(v);   // row_mirror
    return v;
}

__device__ inline float row_sum(float v)
{
    // these forms fold into v_add_f32 with a DPP operand
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
    return v;
}

// Wave totals after row_sum (every lane holds its row's total): rows 0 and 2 are added into
// rows 1 and 3 (row_bcast:15), then rows 0-1 into rows 2-3 (row_bcast:31); lane 63 ends
// with the total of all 64 lanes. Lanes outside the broadcast's target rows add zero.
template <int kCtrl, int kRowMask>
__device__ inline double bcast_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, kRowMask, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, kRowMask, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double rows_to_lane63(double v)
{
    v += bcast_f64<0x142, 0xA>(v);   // row_bcast:15
    v += bcast_f64<0x143, 0xC>(v);   // row_bcast:31
    return v;
}

__device__ inline float rows_to_lane63(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
    return v;
}

__device__ inline float wave_sum(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_lane63(v)), 63));
}

__device__ inline void atomic_add_f32(float *addr, float v)
{
    __hip_atomic_fetch_add(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void atomic_add_f64(double *addr, double v)
{
    __hip_atomic_fetch_add(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace gsx
