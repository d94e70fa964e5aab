// gs_rasterize_fwd / gs_rasterize_bwd: per-tile compositing (Sec. 2.2, eq. 7) and its
// gradients (Sec. 3.1, eqs. 16-21).
//
// One workgroup of 256 lanes (4 wave64) per 16x16 tile, one lane per pixel. The tile's
// depth-ordered list is walked in batches of kBatch splats staged in LDS: each lane
// gathers one 48-byte splat record and stores it pre-scaled so that, per pixel,
//   alpha_raw = o exp(-sigma) = exp2(log2 o + A dx^2 + B dx dy + C dy^2)
// with A = -Y00 log2(e) / 2, B = -Y01 log2(e), C = -Y11 log2(e) / 2 and
// (dx, dy) = Delta = mu' - pixel centre. Every lane of a wave then reads the same LDS
// word (a broadcast, no bank conflicts).
//
// The backward re-walks each pixel's list from its last composited entry, recomputing
// sigma and alpha with the same arithmetic, recovering T by division from T_final
// (eq. 17) and carrying G_S = sum_k dL/dC(k) S(k) (eq. 18 summed over channels). Per
// pair it forms nine terms; they are summed over the wave with DPP (lane 63 holds the
// total), added across the 4 waves in LDS, and flushed to global memory with one
// atomic per term per (tile, splat) after each batch:
//   v = dL/dalpha * alpha        ->  dL/do   = sum v / o
//   v dx, v dy                   ->  dL/dmu' = -Y sum v Delta
//   v dx^2, v dx dy, v dy^2      ->  dL/dY   = -1/2 sum v Delta Delta^T
//   alpha T dL/dC(k)             ->  dL/dc(k)
#include "common.h"

namespace gsx {

constexpr int kBatch = 256;
constexpr float kLog2e = 1.4426950408889634f;

struct TileCtx {
    int tile, start, end;
    int row, col;          // pixel of this lane
    bool inside;
    int64_t pix;           // packed pixel index
};

__device__ inline TileCtx tile_context(const gs_camera *__restrict__ cams, int n_cams,
                                       const int32_t *__restrict__ ranges)
{
    TileCtx t;
    t.tile = blockIdx.x;
    const int c = camera_of_tile(cams, n_cams, t.tile);
    const int local = t.tile - cams[c].tile_offset;
    const int tx_n = cams[c].tiles_x;
    const int ty = local / tx_n, tx = local - ty * tx_n;
    t.row = ty * kTile + (int)(threadIdx.x / kTile);
    t.col = tx * kTile + (int)(threadIdx.x % kTile);
    const int W = cams[c].width, H = cams[c].height;
    t.inside = t.row < H && t.col < W;
    t.pix = cams[c].pixel_offset + (int64_t)t.row * W + t.col;
    t.start = ranges[2 * t.tile];
    t.end = ranges[2 * t.tile + 1];
    return t;
}

// Stage splat ids[k] into slot `slot` of the LDS batch.
struct Stage {
    float4 geo[kBatch];    // mu'x, mu'y, A, B
    float4 geo2[kBatch];   // C, log2 o, c0, c1
    float c2[kBatch];
};

__device__ inline void stage_one(Stage &s, int slot, const float4 *__restrict__ rec, int id)
{
    const float4 r0 = rec[3 * (int64_t)id + 0];
    const float4 r1 = rec[3 * (int64_t)id + 1];
    const float4 r2 = rec[3 * (int64_t)id + 2];
    s.geo[slot] = make_float4(r0.x, r0.y, -0.5f * kLog2e * r0.z, -kLog2e * r0.w);
    s.geo2[slot] = make_float4(-0.5f * kLog2e * r1.x, __log2f(r1.y), r1.z, r1.w);
    s.c2[slot] = r2.x;
}

__device__ inline float alpha_exponent(const float4 &g0, const float4 &g1, float dx, float dy)
{
    return g1.y + dx * (g0.z * dx + g0.w * dy) + g1.x * dy * dy;
}

// ----------------------------------------------------------------------------- forward

__global__ __launch_bounds__(kTilePixels) void raster_fwd_kernel(const float4 *__restrict__ rec,
                                                                 const int32_t *__restrict__ ids,
                                                                 const int32_t *__restrict__ ranges,
                                                                 const gs_camera *__restrict__ cams, int n_cams,
                                                                 gs_params prm, int64_t n_pixels,
                                                                 float *__restrict__ image, float *__restrict__ T_out,
                                                                 int32_t *__restrict__ last_out,
                                                                 int32_t *__restrict__ visited_out)
{
    __shared__ Stage s;
    const TileCtx t = tile_context(cams, n_cams, ranges);
    const float px = (float)t.col + 0.5f, py = (float)t.row + 0.5f;
    float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
    int last = 0, vis = 0;
    bool done = !t.inside;
    for (int b = t.start; b < t.end; b += kBatch) {
        if (__syncthreads_count(done) == kTilePixels) break;
        const int nb = min(kBatch, t.end - b);
        if ((int)threadIdx.x < nb) stage_one(s, threadIdx.x, rec, ids[b + threadIdx.x]);
        __syncthreads();
        if (!done) {
            for (int j = 0; j < nb; ++j) {
                const float4 g0 = s.geo[j], g1 = s.geo2[j];
                const float dx = g0.x - px, dy = g0.y - py;
                const float alpha = fminf(prm.alpha_max, __builtin_amdgcn_exp2f(alpha_exponent(g0, g1, dx, dy)));
                ++vis;
                if (alpha < prm.alpha_min) continue;
                const float Tn = T * (1.f - alpha);
                if (Tn < prm.T_min) { done = true; break; }
                const float w = alpha * T;
                c0 += g1.z * w;
                c1 += g1.w * w;
                c2 += s.c2[j] * w;
                T = Tn;
                last = b - t.start + j + 1;
            }
        }
        __syncthreads();
    }
    if (t.inside) {
        image[t.pix] = c0;
        image[n_pixels + t.pix] = c1;
        image[2 * n_pixels + t.pix] = c2;
        T_out[t.pix] = T;
        last_out[t.pix] = last;
        if (visited_out) visited_out[t.pix] = vis;
    }
}

// ---------------------------------------------------------------------------- backward

struct StageB {
    Stage g;
    int id[kBatch];
    int src[kBatch];
    float opac[kBatch];
    float acc[9][kBatch];
};

__global__ __launch_bounds__(kTilePixels) void raster_bwd_kernel(const float4 *__restrict__ rec,
                                                                 const int32_t *__restrict__ ids,
                                                                 const int32_t *__restrict__ ranges,
                                                                 const gs_camera *__restrict__ cams, int n_cams,
                                                                 gs_params prm, int64_t n_pixels,
                                                                 const float *__restrict__ dL_dimage,
                                                                 const float *__restrict__ T_final,
                                                                 const int32_t *__restrict__ last_in,
                                                                 int64_t n_splats, int64_t n_gauss,
                                                                 float *__restrict__ d_mean2d,
                                                                 float *__restrict__ d_conic,
                                                                 float *__restrict__ d_colors,
                                                                 float *__restrict__ d_opac)
{
    __shared__ StageB s;
    __shared__ int s_maxlast;
    const TileCtx t = tile_context(cams, n_cams, ranges);
    const float px = (float)t.col + 0.5f, py = (float)t.row + 0.5f;
    float gr = 0.f, gg = 0.f, gb = 0.f, T = 1.f;
    int last = 0;
    if (t.inside) {
        gr = dL_dimage[t.pix];
        gg = dL_dimage[n_pixels + t.pix];
        gb = dL_dimage[2 * n_pixels + t.pix];
        T = T_final[t.pix];
        last = last_in[t.pix];
    }
    if (threadIdx.x == 0) s_maxlast = 0;
    __syncthreads();
    if (last > 0) atomicMax(&s_maxlast, last);
    __syncthreads();
    const int maxlast = s_maxlast;
    const int lane = threadIdx.x & (kWave - 1);
    float gS = 0.f;
    for (int bend = t.start + maxlast; bend > t.start; bend -= kBatch) {
        const int bstart = max(t.start, bend - kBatch);
        const int nb = bend - bstart;
        if ((int)threadIdx.x < nb) {
            const int id = ids[bstart + threadIdx.x];
            stage_one(s.g, threadIdx.x, rec, id);
            const float4 r1 = rec[3 * (int64_t)id + 1];
            const float4 r2 = rec[3 * (int64_t)id + 2];
            s.id[threadIdx.x] = id;
            s.opac[threadIdx.x] = r1.y;
            s.src[threadIdx.x] = __float_as_int(r2.z);
#pragma unroll
            for (int q = 0; q < 9; ++q) s.acc[q][threadIdx.x] = 0.f;
        }
        __syncthreads();
        for (int j = nb - 1; j >= 0; --j) {
            const int pos = bstart - t.start + j;   // position in the tile's list
            float v[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) v[q] = 0.f;
            bool contrib = false;
            if (pos < last) {
                const float4 g0 = s.g.geo[j], g1 = s.g.geo2[j];
                const float dx = g0.x - px, dy = g0.y - py;
                const float a_raw = __builtin_amdgcn_exp2f(alpha_exponent(g0, g1, dx, dy));
                const float alpha = fminf(prm.alpha_max, a_raw);
                if (alpha >= prm.alpha_min) {
                    contrib = true;
                    const float r = __builtin_amdgcn_rcpf(1.f - alpha);
                    T = T * r;                                   // T before this splat (eq. 17)
                    const float w = alpha * T;
                    v[6] = w * gr;                               // eq. (16)
                    v[7] = w * gg;
                    v[8] = w * gb;
                    const float gc = gr * g1.z + gg * g1.w + gb * s.g.c2[j];
                    const float dalpha = gc * T - gS * r;        // eq. (18)
                    gS += gc * w;
                    if (a_raw <= prm.alpha_max) {
                        const float vv = dalpha * alpha;         // eq. (19): dalpha/dsigma = -alpha
                        v[0] = vv;
                        v[1] = vv * dx;
                        v[2] = vv * dy;
                        v[3] = vv * dx * dx;
                        v[4] = vv * dx * dy;
                        v[5] = vv * dy * dy;
                    }
                }
            }
            if (__ballot(contrib) != 0) {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const float sum = wave_sum_to_lane63(v[q]);
                    if (lane == kWave - 1) atomicAdd(&s.acc[q][j], sum);
                }
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            const int k = threadIdx.x;
            const float Sv = s.acc[0][k];
            const float c_r = s.acc[6][k], c_g = s.acc[7][k], c_b = s.acc[8][k];
            if (Sv != 0.f || c_r != 0.f || c_g != 0.f || c_b != 0.f) {
                const int id = s.id[k], src = s.src[k];
                const float4 g0 = s.g.geo[k], g1 = s.g.geo2[k];
                const float Y00 = g0.z * (-2.f / kLog2e), Y01 = g0.w * (-1.f / kLog2e), Y11 = g1.x * (-2.f / kLog2e);
                const float Sx = s.acc[1][k], Sy = s.acc[2][k];
                atomic_add_f32(&d_mean2d[id], -(Y00 * Sx + Y01 * Sy));
                atomic_add_f32(&d_mean2d[n_splats + id], -(Y01 * Sx + Y11 * Sy));
                atomic_add_f32(&d_conic[id], -0.5f * s.acc[3][k]);
                atomic_add_f32(&d_conic[n_splats + id], -0.5f * s.acc[4][k]);
                atomic_add_f32(&d_conic[2 * n_splats + id], -0.5f * s.acc[5][k]);
                atomic_add_f32(&d_colors[src], c_r);
                atomic_add_f32(&d_colors[n_gauss + src], c_g);
                atomic_add_f32(&d_colors[2 * n_gauss + src], c_b);
                atomic_add_f32(&d_opac[src], Sv / s.opac[k]);
            }
        }
        __syncthreads();
    }
}

static int check_raster_args(const gs_splats *s, const gs_bins *bins, const gs_camera *cams, int32_t n_cams,
                             const gs_params *prm, int64_t n_pixels)
{
    if (!s || !bins || !cams || !prm || n_cams < 1 || n_pixels < 0 || !s->rec || !bins->ids || !bins->ranges ||
        bins->n_tiles < 0)
        return set_error(GS_ERR_INVALID, "rasterize: null argument or bad size");
    if (((uintptr_t)s->rec) & 15) return set_error(GS_ERR_INVALID, "rasterize: rec must be 16-byte aligned");
    return GS_OK;
}

}  // namespace gsx

using namespace gsx;

extern "C" int gs_rasterize_fwd(const gs_splats *s, const gs_bins *bins, const gs_camera *cams, int32_t n_cams,
                                const gs_params *prm, int64_t n_pixels, float *image, float *T_final,
                                int32_t *last, int32_t *visited, void *stream)
{
    clear_error();
    int rc = check_raster_args(s, bins, cams, n_cams, prm, n_pixels);
    if (rc != GS_OK) return rc;
    if (!image || !T_final || !last) return set_error(GS_ERR_INVALID, "gs_rasterize_fwd: null output");
    if (bins->n_tiles == 0) return GS_OK;
    hipLaunchKernelGGL(raster_fwd_kernel, dim3((unsigned)bins->n_tiles), dim3(kTilePixels), 0, (hipStream_t)stream,
                       (const float4 *)s->rec, bins->ids, bins->ranges, cams, (int)n_cams, *prm, n_pixels, image,
                       T_final, last, visited);
    return check_launch("gs_rasterize_fwd");
}

extern "C" int gs_rasterize_bwd(const gs_splats *s, int64_t n_splats, const gs_bins *bins, const gs_camera *cams,
                                int32_t n_cams, const gs_params *prm, int64_t n_pixels, const float *dL_dimage,
                                const float *T_final, const int32_t *last, float *dL_dmean2d, float *dL_dconic,
                                int64_t n_gaussians, float *dL_dcolors, float *dL_dopac, void *stream)
{
    clear_error();
    int rc = check_raster_args(s, bins, cams, n_cams, prm, n_pixels);
    if (rc != GS_OK) return rc;
    if (!dL_dimage || !T_final || !last || !dL_dmean2d || !dL_dconic || !dL_dcolors || !dL_dopac ||
        n_splats < 0 || n_splats > s->capacity || n_gaussians < 1)
        return set_error(GS_ERR_INVALID, "gs_rasterize_bwd: null argument or bad size");
    if (!(prm->alpha_max < 1.0f))
        return set_error(GS_ERR_INVALID, "gs_rasterize_bwd: alpha_max must be below 1 (eq. 17 divides by 1 - alpha)");
    if (bins->n_tiles == 0) return GS_OK;
    hipLaunchKernelGGL(raster_bwd_kernel, dim3((unsigned)bins->n_tiles), dim3(kTilePixels), 0, (hipStream_t)stream,
                       (const float4 *)s->rec, bins->ids, bins->ranges, cams, (int)n_cams, *prm, n_pixels, dL_dimage,
                       T_final, last, n_splats, n_gaussians, dL_dmean2d, dL_dconic, dL_dcolors, dL_dopac);
    return check_launch("gs_rasterize_bwd");
}
