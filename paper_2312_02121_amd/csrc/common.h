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

__device__ inline float wave_sum(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_lane63(v)), 63));
}

__device__ inline void atomic_add_f32(float *addr, float v)
{
    __hip_atomic_fetch_add(addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace gsx
