// Library runtime: per-thread error state, device check, graph-safe zeroing.
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "common.h"

namespace gsx {

static thread_local int t_hip_error = 0;
static thread_local const char *t_message = "";

int set_error(int code, const char *msg)
{
    t_message = msg;
    return code;
}

void clear_error()
{
    t_hip_error = 0;
    t_message = "";
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return GS_OK;
    t_hip_error = (int)e;
    t_message = what;
    return GS_ERR_HIP;
}

int check_launch(const char *what) { return check_hip(hipGetLastError(), what); }

static gs_tuning g_tuning = {256, 4, 32, 1, 0, 1, 0, 1, 4, 64, 0};

const gs_tuning &current_tuning() { return g_tuning; }

int device_cu_count()
{
    static int cached_dev = -1, cached_cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (dev != cached_dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached_cus = cus;
        cached_dev = dev;
    }
    return cached_cus;
}

unsigned persistent_blocks(int waves_per_block)
{
    return (unsigned)((device_cu_count() * g_tuning.waves_per_cu + waves_per_block - 1) / waves_per_block);
}

__global__ __launch_bounds__(256) void zero_kernel(uint4 *__restrict__ p16, int64_t n16, unsigned char *__restrict__ tail,
                                                   int64_t ntail)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n16; k += stride) p16[k] = make_uint4(0u, 0u, 0u, 0u);
    if (i < ntail) tail[i] = 0;
}

// Zeroes the per-slot gradients dL/dmu' [2][n] and dL/dY [3][n] of the listed slots
// (tiles_touched > 0), the only ones the rasterizer backward adds to and gs_project_bwd reads.
__global__ __launch_bounds__(256) void zero_listed_kernel(const int32_t *__restrict__ tiles, int64_t n,
                                                          double *__restrict__ dm, double *__restrict__ dc)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || tiles[p] <= 0) return;
    dm[p] = 0.0;
    dm[n + p] = 0.0;
    dc[p] = 0.0;
    dc[n + p] = 0.0;
    dc[2 * n + p] = 0.0;
}

}  // namespace gsx

using namespace gsx;

extern "C" int gs_zero_listed_slot_grads(const gs_splats *s, int64_t n_splats, double *dL_dmean2d, double *dL_dconic,
                                         void *stream)
{
    clear_error();
    if (!s || !s->tiles_touched || !dL_dmean2d || !dL_dconic || n_splats < 0 || n_splats > s->capacity)
        return set_error(GS_ERR_INVALID, "gs_zero_listed_slot_grads: null argument or bad size");
    if (n_splats == 0) return GS_OK;
    hipLaunchKernelGGL(zero_listed_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, (hipStream_t)stream,
                       (const int32_t *)s->tiles_touched, n_splats, dL_dmean2d, dL_dconic);
    return check_launch("gs_zero_listed_slot_grads");
}

extern "C" int gs_last_hip_error(void) { return t_hip_error; }

extern "C" const char *gs_last_error_message(void) { return t_message; }

extern "C" int gs_version(void) { return 10000; }

extern "C" int gs_device_check(void)
{
    clear_error();
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc != GS_OK) return rc;
    hipDeviceProp_t prop;
    rc = check_hip(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (rc != GS_OK) return rc;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return set_error(GS_ERR_DEVICE, "device is not gfx950");
    return GS_OK;
}

extern "C" int gs_zero(void *ptr, size_t bytes, void *stream)
{
    clear_error();
    if (bytes == 0) return GS_OK;
    if (!ptr) return set_error(GS_ERR_INVALID, "gs_zero: null pointer");
    // 16-byte stores over the aligned body, byte stores for the unaligned head/tail
    unsigned char *b = (unsigned char *)ptr;
    const uintptr_t mis = ((uintptr_t)b) & 15;
    size_t head = mis ? 16 - mis : 0;
    if (head > bytes) head = bytes;
    hipStream_t st = (hipStream_t)stream;
    if (head) hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, st, (uint4 *)nullptr, 0, b, (int64_t)head);
    const size_t body = bytes - head;
    const int64_t n16 = (int64_t)(body / 16);
    const int64_t tail = (int64_t)(body - (size_t)n16 * 16);
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint4 *)(b + head), n16,
                       b + head + (size_t)n16 * 16, tail);
    return check_launch("gs_zero");
}

// Host-only: sizes and field offsets of the ABI structs, so bindings can check their mirrors.
extern "C" int gs_abi_layout(int64_t *out, int n)
{
    const int64_t v[] = {
        (int64_t)sizeof(gs_camera), (int64_t)offsetof(gs_camera, width), (int64_t)offsetof(gs_camera, near_plane),
        (int64_t)offsetof(gs_camera, gauss_offset), (int64_t)offsetof(gs_camera, pixel_offset),
        (int64_t)offsetof(gs_camera, tile_offset), (int64_t)offsetof(gs_camera, tiles_y),
        (int64_t)sizeof(gs_gaussians), (int64_t)offsetof(gs_gaussians, n),
        (int64_t)sizeof(gs_splats), (int64_t)offsetof(gs_splats, capacity),
        (int64_t)sizeof(gs_params), (int64_t)sizeof(gs_bins), (int64_t)offsetof(gs_bins, capacity),
        (int64_t)offsetof(gs_bins, n_tiles), (int64_t)sizeof(gs_tuning), (int64_t)offsetof(gs_tuning, bwd_segs),
        (int64_t)offsetof(gs_tuning, atomic_lanes), (int64_t)offsetof(gs_tuning, batch),
        (int64_t)offsetof(gs_tuning, big_tiles)};
    const int m = (int)(sizeof(v) / sizeof(v[0]));
    for (int k = 0; k < n && k < m; ++k) out[k] = v[k];
    return m;
}

namespace gsx {
__global__ __launch_bounds__(256) void l2_grad_kernel(const float4 *__restrict__ img, const float4 *__restrict__ tgt,
                                                      int64_t n4, float4 *__restrict__ out,
                                                      const float *__restrict__ img1, const float *__restrict__ tgt1,
                                                      float *__restrict__ out1, int64_t ntail)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) {
        const float4 a = img[i], b = tgt[i];
        out[i] = make_float4(2.f * (a.x - b.x), 2.f * (a.y - b.y), 2.f * (a.z - b.z), 2.f * (a.w - b.w));
    }
    if (i < ntail) out1[i] = 2.f * (img1[i] - tgt1[i]);
}
}  // namespace gsx

// dL/dC of L = sum (C - target)^2 over n floats: dL_dimage = 2 (image - target).
extern "C" int gs_l2_grad(const float *image, const float *target, int64_t n, float *dL_dimage, void *stream)
{
    clear_error();
    if (!image || !target || !dL_dimage || n < 0) return set_error(GS_ERR_INVALID, "gs_l2_grad: bad argument");
    if (n == 0) return GS_OK;
    const bool aligned = ((((uintptr_t)image) | ((uintptr_t)target) | ((uintptr_t)dL_dimage)) & 15) == 0;
    const int64_t n4 = aligned ? n / 4 : 0;
    const int64_t tail = n - 4 * n4;
    const int64_t threads = n4 > tail ? n4 : tail;
    hipLaunchKernelGGL(l2_grad_kernel, dim3(grid_for(threads, 256)), dim3(256), 0, (hipStream_t)stream,
                       (const float4 *)image, (const float4 *)target, n4, (float4 *)dL_dimage, image + 4 * n4,
                       target + 4 * n4, dL_dimage + 4 * n4, tail);
    return check_launch("gs_l2_grad");
}

// ------------------------------------------------------------------------- HIP graphs

struct gs_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" int gs_graph_begin(void *stream)
{
    clear_error();
    if (!stream) return set_error(GS_ERR_INVALID, "gs_graph_begin: capture needs a non-null stream");
    return check_hip(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal),
                     "hipStreamBeginCapture");
}

extern "C" int gs_graph_end(void *stream, gs_graph **out)
{
    clear_error();
    if (!stream || !out) return set_error(GS_ERR_INVALID, "gs_graph_end: null argument");
    *out = nullptr;
    hipGraph_t g = nullptr;
    int rc = check_hip(hipStreamEndCapture((hipStream_t)stream, &g), "hipStreamEndCapture");
    if (rc != GS_OK) return rc;
    hipGraphExec_t e = nullptr;
    rc = check_hip(hipGraphInstantiate(&e, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (rc != GS_OK) {
        (void)hipGraphDestroy(g);
        return rc;
    }
    gs_graph *h = new (std::nothrow) gs_graph{g, e};
    if (!h) {
        (void)hipGraphExecDestroy(e);
        (void)hipGraphDestroy(g);
        return set_error(GS_ERR_INVALID, "gs_graph_end: out of host memory");
    }
    *out = h;
    return GS_OK;
}

extern "C" int gs_graph_launch(gs_graph *graph, void *stream)
{
    clear_error();
    if (!graph) return set_error(GS_ERR_INVALID, "gs_graph_launch: null graph");
    return check_hip(hipGraphLaunch(graph->exec, (hipStream_t)stream), "hipGraphLaunch");
}

extern "C" int gs_graph_destroy(gs_graph *graph)
{
    clear_error();
    if (!graph) return GS_OK;
    const hipError_t e1 = hipGraphExecDestroy(graph->exec);
    const hipError_t e2 = hipGraphDestroy(graph->graph);
    delete graph;
    const int rc = check_hip(e1, "hipGraphExecDestroy");
    return rc != GS_OK ? rc : check_hip(e2, "hipGraphDestroy");
}

extern "C" int gs_set_tuning(const gs_tuning *t)
{
    clear_error();
    if (!t) return set_error(GS_ERR_INVALID, "gs_set_tuning: null argument");
    if (t->split_len < 1 || (t->split_parts != 2 && t->split_parts != 4) || t->waves_per_cu < 4 ||
        t->waves_per_cu > 64 || (t->generate_entries != 0 && t->generate_entries != 1) || t->item_grab < 1 ||
        t->item_grab > 16 || t->prio_len < 0 || (t->bwd_segs != 1 && t->bwd_segs != 2 && t->bwd_segs != 4) ||
        t->atomic_lanes < 1 || t->atomic_lanes > 64 || (t->batch != 32 && t->batch != 64) ||
        (t->big_tiles != 0 && t->big_tiles < 16))
        return set_error(GS_ERR_INVALID, "gs_set_tuning: split_len >= 1, split_parts in {2, 4}, waves_per_cu in "
                                         "[4, 64], generate_entries in {0, 1}, item_grab in [1, 16], prio_len >= 0, "
                                         "bwd_segs in {1, 2, 4}, atomic_lanes in [1, 64], batch in {32, 64}, "
                                         "big_tiles 0 or >= 16");
    g_tuning = *t;
    return GS_OK;
}

extern "C" int gs_get_tuning(gs_tuning *t)
{
    clear_error();
    if (!t) return set_error(GS_ERR_INVALID, "gs_get_tuning: null argument");
    *t = g_tuning;
    return GS_OK;
}
