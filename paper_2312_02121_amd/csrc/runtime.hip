// Library runtime: per-thread error state, device check, graph-safe zeroing.
#include <stddef.h>
#include <string.h>

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

__global__ __launch_bounds__(256) void zero_kernel(uint4 *__restrict__ p16, int64_t n16, unsigned char *__restrict__ tail,
                                                   int64_t ntail)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n16; k += stride) p16[k] = make_uint4(0u, 0u, 0u, 0u);
    if (i < ntail) tail[i] = 0;
}

}  // namespace gsx

using namespace gsx;

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
        (int64_t)offsetof(gs_bins, n_tiles)};
    const int m = (int)(sizeof(v) / sizeof(v[0]));
    for (int k = 0; k < n && k < m; ++k) out[k] = v[k];
    return m;
}
