/*
 * gsplat_mi355x.h -- C ABI of the MI355X (gfx950) differentiable tile rasterizer of
 * 3D Gaussians, following the gsplat mathematical supplement (arXiv 2312.02121).
 *
 * Pipeline (forward, Sec. 2):   gs_project -> gs_bin_and_sort -> gs_rasterize_fwd
 * Pipeline (backward, Sec. 3):  gs_rasterize_bwd -> gs_project_bwd
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every array argument is a DEVICE pointer to caller-owned memory, except the
 *   descriptor structs themselves (gs_gaussians, gs_splats, gs_bins, gs_params),
 *   which are read on the host during the call and may live anywhere. The camera
 *   array `cams` is a device array of gs_camera.
 * - Layouts are structure-of-arrays, component-major float32 planes: a [3][n]
 *   array holds the x plane (n floats), then the y plane, then the z plane.
 * - Every call is stream-ordered and asynchronous on `stream` (a hipStream_t;
 *   NULL = the null stream). No call allocates device memory, synchronises the
 *   host, or writes with hipMemset, so a sequence of calls may be captured in a
 *   HIP graph.
 * - Calls never throw, print or abort. They return a gs_status. On GS_ERR_HIP
 *   the HIP error code is kept for gs_last_hip_error(). gs_last_error_message()
 *   gives a short text for the last failure of the calling thread.
 * - Gradient outputs are ACCUMULATED (+=): zero them first (gs_zero is graph-safe).
 *
 * Readings of the paper that fix the conventions (each is pinned by a CPU test of the
 * FP64 oracle):
 * - quaternions are (w, x, y, z) (Sec. 3.2.1); R(q) is the polynomial of eq. (5) with
 *   R11 = 1 - 2(x^2 + z^2); q is not renormalised unless gs_gaussians.flags has
 *   GS_NORMALIZE_QUATS (an option: R(q / |q|), and gs_project_bwd returns dL/dq through
 *   the normalisation, (dL/dq^ - q^ (q^ . dL/dq^)) / |q|).
 * - mu' follows eq. (2) literally, so a point on the optical axis lands at
 *   (c_x + 1/2, c_y + 1/2); pixel (row i, col j) has centre (j + 1/2, i + 1/2) and
 *   Delta = mu' - pixel centre.
 * - a Gaussian is culled unless near < t_z < far, Sigma' has positive determinant
 *   and its 3-sigma tile box meets the image.
 * - the 3-sigma box has half extents 3 sqrt(Sigma'_00), 3 sqrt(Sigma'_11) (the tight box
 *   of the ellipse), or, with GS_BOX_LAMBDA_MAX, 3 sqrt(lambda_max) on both axes, lambda_max
 *   the largest eigenvalue of Sigma'; tile k covers pixel coordinates [16k, 16k + 16).
 * - alpha = min(alpha_max, o exp(-sigma)); entries with alpha < alpha_min are
 *   skipped; compositing stops before the first entry whose T (1 - alpha) would drop
 *   below T_min (that entry is not composited). alpha_max must lie in (0, 1]; 1 with
 *   alpha_min = T_min = 0 is the literal image formation of eq. (7), in which the kernels
 *   cap alpha at the largest float32 below 1 (1 - alpha >= 2^-24, so the division of
 *   eq. 17 stays defined; only opacities within 6e-8 of 1 are affected).
 * - the image formation of Sec. 2.2 has no background (gs_params.background = 0). A
 *   nonzero background bg is an option: C = sum c alpha T + T_final bg, and the
 *   backward counts bg, with weight T_final, in the colour behind every entry (S of
 *   eq. 18).
 */
#ifndef GSPLAT_MI355X_H
#define GSPLAT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_TILE 16

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID = -1,   /* null pointer, negative size, inconsistent descriptor */
    GS_ERR_CAPACITY = -2,  /* a caller buffer is too small (host-checkable sizes only) */
    GS_ERR_HIP = -3,       /* a HIP call failed; see gs_last_hip_error() */
    GS_ERR_DEVICE = -4     /* the current device is not a gfx950 GPU */
} gs_status;

/*
 * One camera (eq. 1: extrinsics T_cw = [R_cw t_cw; 0 1], intrinsics f, c, image size
 * w x h, clipping planes n, f) plus its place in a batch. 128 bytes; the library
 * reads an array of them from device memory.
 */
typedef struct gs_camera {
    float R[9];             /* R_cw, row-major: camera = R_cw * world + t_cw */
    float t[3];             /* t_cw */
    float fx, fy, cx, cy;   /* focal lengths and principal point, pixels */
    int32_t width, height;  /* w, h */
    float near_plane;       /* n: Gaussians with t_z <= n are culled */
    float far_plane;        /* f: Gaussians with t_z >= f are culled */
    int64_t gauss_offset;   /* first Gaussian of this camera's scene in the gs_gaussians planes */
    int64_t gauss_count;    /* number of Gaussians in that scene */
    int64_t proj_offset;    /* first projected slot: slot = proj_offset + (gaussian - gauss_offset) */
    int64_t pixel_offset;   /* first pixel in the image planes: pixel = offset + row * width + col */
    int32_t tile_offset;    /* first global tile id: tile = offset + ty * tiles_x + tx */
    int32_t tiles_x;        /* ceil(width / 16) */
    int32_t tiles_y;        /* ceil(height / 16) */
    int32_t reserved;
} gs_camera;

/*
 * Gaussian parameters (Sec. 2: mean mu, covariance via scale s and rotation q,
 * colour c, opacity o). Several scenes are concatenated along n; a camera names its
 * scene by (gauss_offset, gauss_count). Read-only device planes.
 */
typedef struct gs_gaussians {
    const float *means;      /* [3][n] */
    const float *quats;      /* [4][n], (w, x, y, z) planes */
    const float *scales;     /* [3][n], linear scales s (eq. 6) */
    const float *colors;     /* [3][n] */
    const float *opacities;  /* [n] */
    int64_t n;
    int32_t flags;           /* projection options: GS_NORMALIZE_QUATS | GS_BOX_LAMBDA_MAX, or 0 */
    int32_t reserved;
} gs_gaussians;

/* gs_gaussians.flags: use q / |q| (in float64) for R(q); a zero quaternion is culled. */
#define GS_NORMALIZE_QUATS 1
/* gs_gaussians.flags: square 3-sigma box of half extent 3 sqrt(lambda_max(Sigma')). */
#define GS_BOX_LAMBDA_MAX 2

/*
 * Projected 2D Gaussians ("splats"), one slot per (camera, Gaussian of its scene):
 * P = sum over cameras of gauss_count. Written by gs_project.
 *   rec[p*12 + 0..1]  mu' (eq. 2), pixels
 *   rec[p*12 + 2..4]  conic Y = Sigma'^{-1} (eq. 4 inverted): Y00, Y01, Y11
 *   rec[p*12 + 5]     opacity o
 *   rec[p*12 + 6..8]  colour c
 *   rec[p*12 + 9]     depth t_z
 *   rec[p*12 + 10]    scene Gaussian index (int32 bits)
 *   rec[p*12 + 11]    camera index (int32 bits)
 * mu', Y and depth are computed in float64 and rounded once to float32. rec is an optional
 * output (NULL: not written): no later step reads it; it states the projection's result in
 * the paper's terms, for inspection and tests.
 */
typedef struct gs_splats {
    float *rec;              /* [P][12], 16-byte aligned, or NULL */
    float *raster;           /* [P][16], 64-byte aligned: compositing record written by gs_project and
                                read by the rasterizer; its layout is private to the library */
    float *depth;            /* [P] t_z (not written for a culled slot) */
    int32_t *rect;           /* [P][4] tile box x0, y0, x1, y1, inclusive, camera-local */
    int32_t *tiles_touched;  /* [P] tiles in the box; 0 = culled */
    int64_t capacity;        /* P */
} gs_splats;

/* Compositing thresholds (see the readings above). Defaults: 1/255, 0.99, 1e-4.
 * background: colour seen through T_final (RGB); zero for the paper's image formation. */
typedef struct gs_params {
    float alpha_min;
    float alpha_max;
    float T_min;
    float background[3];
    int32_t reserved;
} gs_params;

/*
 * Tile-intersection list (Sec. 2.2): one entry per (splat, tile of its box), sorted by
 * key = (global tile << 32) | float32 bits of depth, equal keys in splat order.
 * The rasterizer reads ids and ranges only. With GS_BINS_NO_KEYS in flags the sort does not
 * write the sorted 64-bit keys (ids, ranges and the work list are the same); the keys buffer
 * is still required, as the sort's scratch.
 */
#define GS_BINS_NO_KEYS 1

typedef struct gs_bins {
    uint64_t *keys;          /* [capacity]: the sorted keys, unless flags has GS_BINS_NO_KEYS */
    int32_t *ids;            /* [capacity] splat slot of each entry */
    int32_t *ranges;         /* [n_tiles][2] start, end of each tile's run; empty tile = (0, 0) */
    int32_t *schedule;       /* [gs_schedule_size(n_tiles)] rasterizer work list, written by
                                gs_bin_and_sort; layout private to the library */
    int64_t *counters;       /* [2]: K = total intersections (may exceed capacity), flags
                                (1 = overflow, 2 = sort failure, 4 = camera too wide) */
    int64_t capacity;        /* K_cap, at most 2^31 - 1 */
    int32_t n_tiles;         /* sum over cameras of tiles_x * tiles_y */
    int32_t flags;           /* 0 or GS_BINS_NO_KEYS; other bits are rejected */
} gs_bins;

/*
 * Launch tuning of the rasterizer (not part of the method: results do not depend on it).
 * gs_bin_and_sort builds the work list with split_len and split_parts and picks its first
 * sort pass with generate_entries; the rasterize calls launch with waves_per_cu and
 * split_priority. The setting is process-wide and is
 * read when a call is made, so a captured graph keeps the tuning it was captured with.
 */
typedef struct gs_tuning {
    int32_t split_len;       /* tiles with at least this many list entries become split_parts
                                work items; >= 1 (a value above any list length disables it) */
    int32_t split_parts;     /* 2 (16x8-pixel halves, 2 pixels per lane) or
                                4 (16x4-pixel quarters, 1 pixel per lane) */
    int32_t waves_per_cu;    /* persistent grid: waves launched per compute unit, 4..64 */
    int32_t split_priority;  /* nonzero: a wave raises its issue priority on a split item */
    int32_t generate_entries;/* nonzero: the first tile-sort pass generates the list entries from
                                the boxes itself instead of reading them from an emitted list
                                (less traffic when splats cover many tiles) */
    int32_t item_grab;       /* work items a wave takes from the work list per atomic on its
                                counter, 1..16 (fewer atomics on one address when items are
                                many and short; more imbalance at the end of the list) */
    int32_t prio_len;        /* a wave also raises its issue priority on an unsplit tile whose
                                walk has at least this many entries (level 1; level 2 from
                                twice as many; split items take level 3); 0: never. Long walks
                                are the end of the launch: priority keeps them near full speed
                                while the SIMD is shared */
    int32_t bwd_segs;        /* 1, 2 or 4: the fused kernel walks the backward of a split tile's
                                part as this many list segments, one work item each (every
                                such item repeats the part's forward), so that the longest
                                walks, the end of the launch, are shorter */
    int32_t atomic_lanes;    /* 1..64: in the backward, a splat whose pixels with a nonzero
                                alpha sit in at most this many lanes of a wave is summed with
                                LDS atomics from those lanes; otherwise the wave sums it with
                                DPP row operations (cheaper for large splats) */
    int32_t batch;           /* 32 or 64: list entries a wave stages in LDS per batch (one per
                                lane; gradients are moved to memory once per batch) */
    int32_t big_tiles;       /* 0, or >= 16: gs_bin_and_sort lists a splat whose box has more than
                                this many tiles by a per-tile merge instead of sorting its entries
                                by tile (the list is the same; for calls of at most 64 cameras,
                                with tile coordinates below 65536, else flag 2). Pays off when a
                                few splats cover most tiles of a view */
} gs_tuning;

/* ------------------------------------------------------------------------- utilities */

/* Returns GS_OK if the current HIP device is a gfx950 GPU, GS_ERR_DEVICE otherwise. */
int gs_device_check(void);

/* HIP error code of the last GS_ERR_HIP returned on this thread (0 if none). */
int gs_last_hip_error(void);

/* Static text describing the last failure on this thread ("" if none). */
const char *gs_last_error_message(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int gs_version(void);

/* Sets the process-wide launch tuning (see gs_tuning). GS_ERR_INVALID for values out of
 * range. Not synchronised with calls running on other host threads. */
int gs_set_tuning(const gs_tuning *t);

/* Reads the current launch tuning into *t. */
int gs_get_tuning(gs_tuning *t);

/*
 * Polls a look-back wait inside gs_bin_and_sort's single-pass sort launches makes before it
 * gives up (default 2^20), on the current device. A wait that gives up sets counters[1] & 2
 * and the call builds no list (every range empty); every kernel still ends normally. A
 * negative value makes every look-back give up at once: it drives that failure path on
 * purpose, for tests of the caller's error handling. Synchronous (a copy to device memory);
 * not to be called while binning runs.
 */
int gs_set_sort_wait_limit(int32_t polls);

/*
 * Measurement aid: with counts (device memory, two uint64, caller-zeroed) the rasterizer
 * kernels add to counts[0] the Gaussian-pixel pairs their forward walks execute (list
 * slots stepped through x pixels of the wave, padding slots and finished pixels included,
 * left-out records not) and to counts[1] those of their backward walks; NULL (the default)
 * turns counting off. Applies to launches made after the call on the current device.
 * Synchronous (a copy to device memory).
 */
int gs_set_work_counter(unsigned long long *counts);

/* Zeroes `bytes` bytes at device pointer `ptr` with a kernel (graph-capturable). */
int gs_zero(void *ptr, size_t bytes, void *stream);

/*
 * Zeroes dL_dmean2d [2][n_splats] and dL_dconic [3][n_splats] (float64, the per-slot
 * gradients of gs_rasterize_bwd / gs_rasterize_fused_l2) at the slots the projection listed
 * (s->tiles_touched > 0) only: those are the only slots the rasterizer adds to and
 * gs_project_bwd reads, so this is enough before a backward that follows the same
 * projection. Culled slots keep whatever they held. Graph-capturable.
 */
int gs_zero_listed_slot_grads(const gs_splats *s, int64_t n_splats, double *dL_dmean2d, double *dL_dconic,
                              void *stream);

/*
 * Host-only query of the ABI struct layout, for bindings that mirror the structs:
 * writes up to n int64 values (sizeof and selected offsetof of gs_camera,
 * gs_gaussians, gs_splats, gs_params, gs_bins, in the order of the implementation)
 * to out and returns how many values exist. Touches no device.
 */
int gs_abi_layout(int64_t *out, int n);

/*
 * Gradient of the L2 image loss L = sum (C - target)^2 used by the training step:
 * dL_dimage[i] = 2 (image[i] - target[i]) for i < n. Not part of the paper's method.
 */
int gs_l2_grad(const float *image, const float *target, int64_t n, float *dL_dimage, void *stream);

/* --------------------------------------------------------------------- forward (Sec. 2) */

/*
 * Sec. 2.1 (eqs. 1-6) and the 3-sigma box of Sec. 2.2, for every (camera, Gaussian)
 * pair: R(q), Sigma = R S S^T R^T, t = T_cw [mu; 1], t' = P t, mu', J, Sigma' =
 * J R_cw Sigma R_cw^T J^T, Y = Sigma'^{-1}, box and tile count.
 * g: Gaussian planes. cams: device array of n_cams cameras whose proj_offset ranges
 * tile [0, n_splats). out: splat buffers of capacity >= n_splats; tiles_touched is written
 * for every slot, the other fields only for slots with tiles_touched > 0 (a culled slot's
 * record, depth and box are left as they were).
 * Errors: GS_ERR_INVALID for null pointers (other than out->rec), n_cams < 1,
 * n_splats < 0 or n_splats > out->capacity.
 */
int gs_project(const gs_gaussians *g, const gs_camera *cams, int32_t n_cams, int64_t n_splats,
               gs_splats *out, void *stream);

/*
 * Per-stage form (the projection of Sec. 2.1 and the rasterizer of Sec. 2.2 as separate
 * differentiable steps): writes the splats gs_bin_and_sort and the rasterizer read from
 * given 2D quantities instead of projecting. Per slot p (slots as in gs_project):
 *   mean2d [2][n_splats] mu', conic [3][n_splats] Y = (Y00, Y01, Y11), depth [n_splats],
 *   valid [n_splats] int32 (0: the slot stays culled, e.g. where gs_project culled it).
 * Colours and opacities come from the slot's scene Gaussian in g (means, quats, scales are
 * not read). The 3-sigma box is decided on Sigma' = Y^-1, formed in float64 from the given
 * float32 Y, with the box option of g->flags; a slot is culled where Y is not positive
 * definite or its box misses the image. The rasterizer's gradients dL/dmu' and dL/dY then
 * refer to these inputs. out->rec is not written. Errors: GS_ERR_INVALID for null pointers,
 * bad sizes or misaligned planes.
 */
int gs_splats_from_2d(const gs_gaussians *g, const gs_camera *cams, int32_t n_cams, int64_t n_splats,
                      const float *mean2d, const float *conic, const float *depth, const int32_t *valid,
                      gs_splats *out, void *stream);

/* Number of int32 entries of gs_bins.schedule for n_tiles tiles. */
int64_t gs_schedule_size(int32_t n_tiles);

/* Bytes of workspace gs_bin_and_sort needs for n_splats splats and a list capacity. */
size_t gs_bin_and_sort_workspace_size(int64_t n_splats, int64_t capacity, int32_t n_tiles);

/*
 * Sec. 2.2: duplicate each splat once per tile of its box, sort the entries by
 * (tile, depth) with ties in splat order -- the order of one stable LSD radix sort of the
 * 64-bit keys -- and find each tile's [start, end), then write the rasterizer's work list
 * (tiles in decreasing list length, long ones split into four parts). The sort is done as
 * a stable depth sort of the splats followed by a stable tile-id sort of the entries
 * emitted in depth order, which yields the same list (with gs_tuning.big_tiles, splats
 * covering more tiles skip the tile sort and are merged into each tile's run by depth rank,
 * again the same list); the ranges come from each tile's list length, counted from the
 * boxes (a 2D difference array per camera). K is written to
 * bins->counters[0]; if K exceeds bins->capacity the list is not built (every tile's
 * range is empty, so a rasterize call made before the caller looks renders nothing and
 * reads nothing from the list), counters[1] is set to 1, and the caller regrows and calls
 * again. counters[1] & 2 means a
 * wait inside the single-pass sort gave up after its spin limit, or the counted lengths
 * disagree with K (the list is invalid and every range empty; this indicates a fault, not
 * a capacity problem); counters[1] & 4: a camera has more than 8192 tiles in a row (wider
 * than 131072 pixels), which is not supported (nothing is listed). workspace: device
 * memory of at least gs_bin_and_sort_workspace_size() bytes, 256-byte aligned, contents
 * free on entry and exit. cams: as for gs_project.
 * Concurrency: the single-pass sort launches deal their chunks to a grid of blocks that is
 * resident all at once and whose blocks wait on each other (each wait bounded by a spin
 * limit). No other kernel may run on the device while the call's launches do: a concurrent
 * kernel can hold back some of those blocks until the waits give up, which sets
 * counters[1] & 2 (the list is then invalid, every range empty). Issue the call on a
 * stream that nothing else runs beside, or after a device-wide ordering point.
 * Errors: GS_ERR_INVALID (null pointers, capacity outside [1, 2^31 - 1], n_splats outside
 * [0, 2^31 - 1], more cameras than tiles, workspace not 256-byte aligned), GS_ERR_CAPACITY
 * (workspace too small).
 */
int gs_bin_and_sort(const gs_splats *s, int64_t n_splats, const gs_camera *cams, int32_t n_cams,
                    gs_bins *bins, void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of the static workspace of gs_bin_and_sort_static (per GPU). */
#define GS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/*
 * gs_bin_and_sort without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same inputs, outputs, list, ranges, work list and flags as gs_bin_and_sort.
 * The workspace is a static array of GS_STATIC_WORKSPACE_BYTES inside the library, one per
 * GPU, which each GPU holds until the process ends; the call makes no allocation of its own.
 * It serves every call whose gs_bin_and_sort_workspace_size(n_splats, capacity, n_tiles)
 * fits in it (for example 1M splats with a 1.6M-entry list at 1920x1080). The array keeps
 * the last call's contents; each call clears what it needs cleared. Calls that overlap on
 * one GPU (on different streams, or from several host threads) share the array and race:
 * the caller must order them. The concurrency rule of gs_bin_and_sort applies as well.
 * Errors: as gs_bin_and_sort; GS_ERR_CAPACITY when the call needs more workspace than the
 * static array holds (nothing is launched), GS_ERR_HIP if the array's device address
 * cannot be obtained.
 */
int gs_bin_and_sort_static(const gs_splats *s, int64_t n_splats, const gs_camera *cams, int32_t n_cams,
                           gs_bins *bins, void *stream);

/*
 * Sec. 2.2, eq. (7): per pixel, composite its tile's list front to back with online
 * transmittance. A persistent launch takes work items (whole 16x16 tiles, or 16x4 quarters
 * of long-list tiles) from the work list gs_bin_and_sort wrote, longest first.
 * Outputs over the packed pixels of all cameras (n_pixels = sum of width * height):
 *   image   [3][n_pixels]  C (plus T_final times prm->background)
 *   T_final [n_pixels]     T after the last composited entry
 *   last    [n_pixels]     1 + list position (within the tile's run) of the last
 *                          composited entry, 0 if none: where the backward starts
 *   visited [n_pixels]     optional (NULL to skip): entries whose alpha was evaluated,
 *                          including a terminating entry
 * Errors: GS_ERR_INVALID for null pointers or inconsistent sizes.
 */
int gs_rasterize_fwd(const gs_splats *s, const gs_bins *bins, const gs_camera *cams, int32_t n_cams,
                     const gs_params *prm, int64_t n_pixels, float *image, float *T_final,
                     int32_t *last, int32_t *visited, void *stream);

/* -------------------------------------------------------------------- backward (Sec. 3) */

/*
 * Sec. 3.1 (eqs. 16-21): walk each pixel's list back to front from `last`, recover
 * T by division from T_final (eq. 17), recompute sigma and alpha, and accumulate:
 *   dL_dmean2d [2][n_splats]    dL/dmu' (float64)
 *   dL_dconic  [3][n_splats]    dL/dY (float64) as the (0,0), (0,1), (1,1) entries of the
 *                               full-matrix gradient (the off-diagonal is not doubled)
 *   dL_dcolors [3][n_gaussians] dL/dc per scene Gaussian
 *   dL_dopac   [n_gaussians]    dL/do per scene Gaussian
 * dL_dimage [3][n_pixels]; T_final and last from gs_rasterize_fwd with the same
 * inputs (and the same prm, whose background enters through T_final). Gradients of
 * clamped alphas (o exp(-sigma) > alpha_max) reach only c.
 * Outputs are accumulated; zero them first. dL/dmu' and dL/dY are float64 because
 * gs_project_bwd multiplies them by Y on both sides (dL/dSigma' = -Y dL/dY Y): for a
 * needle-like splat float32 rounding of dL/dY, scaled by the square of Y's largest
 * eigenvalue, would dominate the gradient along the splat's thin axis.
 * Errors: GS_ERR_INVALID for null pointers, bad sizes, or alpha_max outside (0, 1].
 */
int gs_rasterize_bwd(const gs_splats *s, int64_t n_splats, const gs_bins *bins, const gs_camera *cams,
                     int32_t n_cams, const gs_params *prm, int64_t n_pixels, const float *dL_dimage,
                     const float *T_final, const int32_t *last, double *dL_dmean2d, double *dL_dconic,
                     int64_t n_gaussians, float *dL_dcolors, float *dL_dopac, void *stream);

/*
 * Fused training step over a batch of cameras: for every work item (a tile, or a quarter
 * of a long-list tile, of any camera) the forward of eq. (7), the gradient of the L2
 * image loss L = sum (C - target)^2, dL/dC = 2 (C - target), and the backward of
 * Sec. 3.1 run back to back inside one persistent launch, so the image, T and `last`
 * stay in registers. C includes the background term of prm. target [3][n_pixels].
 * image: optional (NULL) output of C. loss:
 * optional (NULL) device float to which L is added. When bins->counters[1] is nonzero
 * (gs_bin_and_sort built no list: overflow or a failed sort) the launch writes NaN to
 * *loss and nothing else, so a caller that does not synchronise after binning still sees
 * that the step is void. Gradient outputs and errors as for gs_rasterize_bwd
 * (accumulated; zero them first); bins->counters must not be NULL.
 */
int gs_rasterize_fused_l2(const gs_splats *s, int64_t n_splats, const gs_bins *bins, const gs_camera *cams,
                          int32_t n_cams, const gs_params *prm, int64_t n_pixels, const float *target,
                          float *image, float *loss, double *dL_dmean2d, double *dL_dconic,
                          int64_t n_gaussians, float *dL_dcolors, float *dL_dopac, void *stream);

/*
 * Sec. 3.2 and 3.2.1 (eqs. 22-31): from dL/dmu' and dL/dY of each visible splat,
 * dL/dSigma' = -Y dL/dY Y, the mean route of eq. (23) (second row with h), the
 * covariance route through T = J R_cw and dJ/dt, then dL/dmu = R_cw^T dL/dt,
 * dL/dSigma = T^T dL/dSigma' T, dL/dM = 2 dL/dSigma M, dL/dR = dL/dM S^T,
 * dL/dS = R^T dL/dM, dL/dq = <dL/dR, dR/dq>, dL/ds_j = (dL/dS)_jj.
 * Scene gradients [3][n] means, [3][n] scales, [4][n] quats are accumulated over
 * cameras. dL_dcampose: optional (NULL to skip) [n_cams][12] row-major 3x4 gradient of
 * [R_cw | t_cw] per camera (eq. 28 plus the R_cw term through T = J R_cw).
 */
int gs_project_bwd(const gs_gaussians *g, const gs_camera *cams, int32_t n_cams, const gs_splats *s,
                   int64_t n_splats, const double *dL_dmean2d, const double *dL_dconic,
                   float *dL_dmeans, float *dL_dscales, float *dL_dquats, float *dL_dcampose,
                   void *stream);

/* ------------------------------------------------------------------------ HIP graphs */

/*
 * A captured sequence of calls, replayable with one launch. Every call above is
 * capture-safe (no allocation, no host synchronisation, no hipMemset), so a training
 * step (project, bin_and_sort, zero, fused rasterization, project_bwd) can be captured
 * once and replayed while the buffers it names stay allocated. The list capacity is fixed
 * at capture time: read bins->counters[1] after a replay and recapture with larger
 * buffers if it is set.
 */
typedef struct gs_graph gs_graph;

/* Starts capturing `stream` (a non-null hipStream_t) in thread-local mode. */
int gs_graph_begin(void *stream);

/* Ends the capture of `stream` and instantiates it; *out receives the graph. */
int gs_graph_end(void *stream, gs_graph **out);

/* Replays the graph on `stream`. */
int gs_graph_launch(gs_graph *graph, void *stream);

/* Releases the graph. */
int gs_graph_destroy(gs_graph *graph);

#ifdef __cplusplus
}
#endif

#endif /* GSPLAT_MI355X_H */
