// gs_project: projection of 3D Gaussians (Sec. 2.1, eqs. 1-6) and their 3-sigma tile
// boxes (Sec. 2.2). One thread per scene Gaussian, projected into every camera that views it.
//
// The arithmetic runs in float64 without FMA contraction and every sum is evaluated
// left to right in the order the equations are written (matrix products row by
// column). mu', Y = Sigma'^{-1} and t_z are rounded once to float32 when stored, and
// the tile box is decided on the float64 values. Projection is HBM-bound (40 bytes in,
// ~84 bytes out per slot), so the float64 arithmetic costs nothing measurable and
// makes the discrete outputs (box, tile count) reproducible.
#include "common.h"

namespace gsx {

// Tile box of the 3-sigma ellipse of Sigma' = (C00, C01; C01, C11) around mu' on the 16x16
// grid of the camera (Sec. 2.2): tight axis-aligned half extents 3 sqrt(C00), 3 sqrt(C11),
// or with GS_BOX_LAMBDA_MAX a square from the largest eigenvalue. False when it misses the
// image; otherwise box (clamped to the image) and its tile count.
__device__ inline bool splat_box(double mu0, double mu1, double C00, double C01, double C11, const gs_camera &cam,
                                 int flags, int4 &box, int32_t &tiles)
{
#pragma clang fp contract(off)
    double ex = 3.0 * sqrt(C00), ey = 3.0 * sqrt(C11);
    if (flags & GS_BOX_LAMBDA_MAX) {
        // square from the largest eigenvalue of Sigma' (contains the tight box)
        const double h = (C00 - C11) / 2.0;
        const double lmax = (C00 + C11) / 2.0 + sqrt(h * h + C01 * C01);
        ex = ey = 3.0 * sqrt(lmax);
    }
    const double TX = (double)cam.tiles_x, TY = (double)cam.tiles_y;
    double x0 = floor((mu0 - ex) / 16.0), x1 = floor((mu0 + ex) / 16.0);
    double y0 = floor((mu1 - ey) / 16.0), y1 = floor((mu1 + ey) / 16.0);
    if (!(x1 >= 0.0 && y1 >= 0.0 && x0 <= TX - 1.0 && y0 <= TY - 1.0)) return false;
    x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
    x1 = fmin(x1, TX - 1.0); y1 = fmin(y1, TY - 1.0);
    box = make_int4((int)x0, (int)y0, (int)x1, (int)y1);
    tiles = (box.z - box.x + 1) * (box.w - box.y + 1);
    return true;
}

// Compositing record of a splat from its float32 mu', conic Y, opacity and colour.
__device__ inline RasterRec make_record(float mx, float my, float y00, float y01, float y11, float o, float c0,
                                        float c1, float c2, int src, int slot)
{
    RasterRec rr;
    rr.mx = mx;
    rr.my = my;
    rr.lo = o > 0.f ? log2((double)o) : -INFINITY;
    rr.A = -0.5 * kLog2eD * (double)y00;
    rr.B = -kLog2eD * (double)y01;
    rr.C = -0.5 * kLog2eD * (double)y11;
    rr.c0 = c0;
    rr.c1 = c1;
    rr.c2 = c2;
    rr.o = o;
    rr.src = src;
    rr.slot = slot;
    return rr;
}

// One scene Gaussian as the projection reads it: mean, (normalised) quaternion and scale in
// float64, whether all of them are finite, and Sigma = M M^T with M = R(q) S (eqs. 5, 6), which
// does not depend on the camera.
struct GaussIn {
    double mx, my, mz;
    bool finite;
    double S00, S01, S02, S11, S12, S22;
};

__device__ inline GaussIn load_gaussian(const gs_gaussians &g, int64_t i)
{
#pragma clang fp contract(off)
    const int64_t n = g.n;
    GaussIn gi;
    gi.mx = g.means[i];
    gi.my = g.means[n + i];
    gi.mz = g.means[2 * n + i];
    double qw = g.quats[i], qx = g.quats[n + i], qy = g.quats[2 * n + i], qz = g.quats[3 * n + i];
    if (g.flags & GS_NORMALIZE_QUATS) {
        // q / |q|; a zero or non-finite q gives a non-finite result, which is culled
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw = qw / qn;
        qx = qx / qn;
        qy = qy / qn;
        qz = qz / qn;
    }
    const double s0 = g.scales[i], s1 = g.scales[n + i], s2 = g.scales[2 * n + i];
    gi.finite = isfinite(gi.mx) && isfinite(gi.my) && isfinite(gi.mz) && isfinite(qw) && isfinite(qx) &&
                isfinite(qy) && isfinite(qz) && isfinite(s0) && isfinite(s1) && isfinite(s2);
    // R(q), eq. (5) with R11 = 1 - 2(x^2 + z^2); M = R S; Sigma = M M^T (eq. 6)
    const double q00 = 1.0 - 2.0 * (qy * qy + qz * qz), q01 = 2.0 * (qx * qy - qw * qz), q02 = 2.0 * (qx * qz + qw * qy);
    const double q10 = 2.0 * (qx * qy + qw * qz), q11 = 1.0 - 2.0 * (qx * qx + qz * qz), q12 = 2.0 * (qy * qz - qw * qx);
    const double q20 = 2.0 * (qx * qz - qw * qy), q21 = 2.0 * (qy * qz + qw * qx), q22 = 1.0 - 2.0 * (qx * qx + qy * qy);
    const double M00 = q00 * s0, M01 = q01 * s1, M02 = q02 * s2;
    const double M10 = q10 * s0, M11 = q11 * s1, M12 = q12 * s2;
    const double M20 = q20 * s0, M21 = q21 * s1, M22 = q22 * s2;
    gi.S00 = M00 * M00 + M01 * M01 + M02 * M02;
    gi.S01 = M00 * M10 + M01 * M11 + M02 * M12;
    gi.S02 = M00 * M20 + M01 * M21 + M02 * M22;
    gi.S11 = M10 * M10 + M11 * M11 + M12 * M12;
    gi.S12 = M10 * M20 + M11 * M21 + M12 * M22;
    gi.S22 = M20 * M20 + M21 * M21 + M22 * M22;
    return gi;
}

// The projection of Gaussian i (loaded as gi) through camera c into its slot p.
__device__ inline void project_slot(const gs_gaussians &g, const gs_camera &cam, int c, int64_t i, int64_t p,
                                    const GaussIn &gi, float4 *__restrict__ rec, RasterRec *__restrict__ rrec,
                                    float *__restrict__ depth_out, int4 *__restrict__ rect_out,
                                    int32_t *__restrict__ tiles_out)
{
#pragma clang fp contract(off)
    const int64_t n = g.n;
    const double mx = gi.mx, my = gi.my, mz = gi.mz;
    // t = T_cw [mu; 1]
    const double R00 = cam.R[0], R01 = cam.R[1], R02 = cam.R[2];
    const double R10 = cam.R[3], R11 = cam.R[4], R12 = cam.R[5];
    const double R20 = cam.R[6], R21 = cam.R[7], R22 = cam.R[8];
    const double tx = R00 * mx + R01 * my + R02 * mz + (double)cam.t[0];
    const double ty = R10 * mx + R11 * my + R12 * mz + (double)cam.t[1];
    const double tz = R20 * mx + R21 * my + R22 * mz + (double)cam.t[2];
    // depth keys are the float bits of t_z, which order depths correctly only when t_z > 0:
    // a near plane at or behind the camera still culls t_z <= 0
    bool visible = gi.finite && isfinite(tx) && isfinite(ty) && tz > (double)cam.near_plane && tz > 0.0 &&
                   tz < (double)cam.far_plane;

    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    RasterRec rr = {};
    int4 box = make_int4(0, 0, 0, 0);
    int32_t tiles = 0;
    float dep = 0.f;

    if (visible) {
        // t' = P t with P of eq. (1); mu' of eq. (2)
        const double w = (double)cam.width, h = (double)cam.height;
        const double fx = cam.fx, fy = cam.fy;
        const double tpx = (2.0 * fx / w) * tx;
        const double tpy = (2.0 * fy / h) * ty;
        const double mu0 = (w * tpx / tz + 1.0) / 2.0 + (double)cam.cx;
        const double mu1 = (h * tpy / tz + 1.0) / 2.0 + (double)cam.cy;

        // J of eq. (3) and T = J R_cw
        const double J00 = fx / tz, J02 = -(fx * tx) / (tz * tz);
        const double J11 = fy / tz, J12 = -(fy * ty) / (tz * tz);
        const double T00 = J00 * R00 + J02 * R20, T01 = J00 * R01 + J02 * R21, T02 = J00 * R02 + J02 * R22;
        const double T10 = J11 * R10 + J12 * R20, T11 = J11 * R11 + J12 * R21, T12 = J11 * R12 + J12 * R22;

        // Sigma' = (T Sigma) T^T, eq. (4)
        const double U00 = T00 * gi.S00 + T01 * gi.S01 + T02 * gi.S02;
        const double U01 = T00 * gi.S01 + T01 * gi.S11 + T02 * gi.S12;
        const double U02 = T00 * gi.S02 + T01 * gi.S12 + T02 * gi.S22;
        const double U10 = T10 * gi.S00 + T11 * gi.S01 + T12 * gi.S02;
        const double U11 = T10 * gi.S01 + T11 * gi.S11 + T12 * gi.S12;
        const double U12 = T10 * gi.S02 + T11 * gi.S12 + T12 * gi.S22;
        const double C00 = U00 * T00 + U01 * T01 + U02 * T02;
        const double C01 = U00 * T10 + U01 * T11 + U02 * T12;
        const double C11 = U10 * T10 + U11 * T11 + U12 * T12;
        const double det = C00 * C11 - C01 * C01;

        visible = isfinite(C00) && isfinite(C01) && isfinite(C11) && det > 0.0 && C00 > 0.0 && C11 > 0.0;
        const double Y00 = C11 / det, Y01 = -C01 / det, Y11 = C00 / det;
        visible = visible && isfinite(mu0) && isfinite(mu1) && isfinite(Y00) && isfinite(Y01) && isfinite(Y11);

        if (visible) {
            // axis-aligned box of the 3-sigma ellipse on the 16x16 tile grid
            visible = splat_box(mu0, mu1, C00, C01, C11, cam, g.flags, box, tiles);
            if (visible) {
                dep = (float)tz;
                const float y00 = (float)Y00, y01 = (float)Y01, y11 = (float)Y11;
                const float o = g.opacities[i];
                r0 = make_float4((float)mu0, (float)mu1, y00, y01);
                r1 = make_float4(y11, o, g.colors[i], g.colors[n + i]);
                r2 = make_float4(g.colors[2 * n + i], dep, __int_as_float((int)i), __int_as_float(c));
                rr = make_record(r0.x, r0.y, y00, y01, y11, o, r1.z, r1.w, r2.x, (int)i, (int)p);
            }
        }
    }
    // a culled slot (tiles_touched = 0) is never listed, so only its count is written
    tiles_out[p] = tiles;
    if (tiles > 0) {
        if (rec) {   // optional output, uniform
            rec[3 * p + 0] = r0;
            rec[3 * p + 1] = r1;
            rec[3 * p + 2] = r2;
        }
        rrec[p] = rr;
        depth_out[p] = dep;
        rect_out[p] = box;
    }
}

// Gaussian-major: one thread per scene Gaussian, which is read once and projected into the
// slot of every camera that views its scene (cameras hold contiguous slices of the Gaussian
// planes and of the slots). A wave holds 64 consecutive Gaussians, so each camera's slots are
// written 64 at a time, coalesced, and a batch of views reads the Gaussians once instead of
// once per view.
__global__ __launch_bounds__(256) void project_kernel(gs_gaussians g, const gs_camera *__restrict__ cams,
                                                      int n_cams, int64_t n_splats, float4 *__restrict__ rec,
                                                      RasterRec *__restrict__ rrec, float *__restrict__ depth_out,
                                                      int4 *__restrict__ rect_out, int32_t *__restrict__ tiles_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const GaussIn gi = load_gaussian(g, i);
    for (int c = 0; c < n_cams; ++c) {
        const gs_camera &cam = cams[c];
        const int64_t k = i - cam.gauss_offset;
        if (k < 0 || k >= cam.gauss_count) continue;
        const int64_t p = cam.proj_offset + k;
        if (p >= n_splats) continue;
        project_slot(g, cam, c, i, p, gi, rec, rrec, depth_out, rect_out, tiles_out);
    }
}

// Splats from given 2D quantities (the per-stage form): mu' [2][n_splats], Y [3][n_splats]
// and depth [n_splats] per slot, colours and opacities from the slot's scene Gaussian. The
// slot keeps its projection only where valid[p] != 0; Sigma' = Y^-1 in float64 from the
// float32 conic decides the box, as the projection decides it from its own Sigma'.
__global__ __launch_bounds__(256) void splats_from_2d_kernel(gs_gaussians g, const gs_camera *__restrict__ cams,
                                                             int n_cams, int64_t n_splats,
                                                             const float *__restrict__ mean2d,
                                                             const float *__restrict__ conic,
                                                             const float *__restrict__ depth_in,
                                                             const int32_t *__restrict__ valid,
                                                             RasterRec *__restrict__ rrec, float *__restrict__ depth_out,
                                                             int4 *__restrict__ rect_out, int32_t *__restrict__ tiles_out)
{
#pragma clang fp contract(off)
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_splats) return;
    const int c = camera_of_splat(cams, n_cams, p);
    const gs_camera &cam = cams[c];
    const int64_t n = g.n;
    const int64_t i = cam.gauss_offset + (p - cam.proj_offset);
    const float m0 = mean2d[p], m1 = mean2d[n_splats + p];
    const float y00 = conic[p], y01 = conic[n_splats + p], y11 = conic[2 * n_splats + p];
    const double Y00 = y00, Y01 = y01, Y11 = y11;
    const double det = Y00 * Y11 - Y01 * Y01;
    const double C00 = Y11 / det, C01 = -Y01 / det, C11 = Y00 / det;
    int4 box = make_int4(0, 0, 0, 0);
    int32_t tiles = 0;
    // a depth that is not positive and finite cannot be a depth key (float bits order only
    // positive values): the slot is culled
    const float dep = depth_in[p];
    bool visible = valid[p] != 0 && isfinite((double)m0) && isfinite((double)m1) && isfinite(det) && det > 0.0 &&
                   Y00 > 0.0 && Y11 > 0.0 && isfinite(C00) && isfinite(C01) && isfinite(C11) && dep > 0.0f &&
                   isfinite(dep);
    if (visible) visible = splat_box(m0, m1, C00, C01, C11, cam, g.flags, box, tiles);
    tiles_out[p] = visible ? tiles : 0;
    if (visible) {
        const float o = g.opacities[i];
        rrec[p] = make_record(m0, m1, y00, y01, y11, o, g.colors[i], g.colors[n + i], g.colors[2 * n + i], (int)i,
                              (int)p);
        depth_out[p] = dep;
        rect_out[p] = box;
    }
}

}  // namespace gsx

using namespace gsx;

extern "C" int gs_splats_from_2d(const gs_gaussians *g, const gs_camera *cams, int32_t n_cams, int64_t n_splats,
                                 const float *mean2d, const float *conic, const float *depth, const int32_t *valid,
                                 gs_splats *out, void *stream)
{
    clear_error();
    if (!g || !cams || !out || n_cams < 1 || n_splats < 0)
        return set_error(GS_ERR_INVALID, "gs_splats_from_2d: null argument or bad size");
    if (n_splats > out->capacity)
        return set_error(GS_ERR_INVALID, "gs_splats_from_2d: n_splats exceeds splat capacity");
    if (n_splats == 0) return GS_OK;
    if (!mean2d || !conic || !depth || !valid || !g->colors || !g->opacities || g->n < 1 || !out->raster ||
        !out->depth || !out->rect || !out->tiles_touched)
        return set_error(GS_ERR_INVALID, "gs_splats_from_2d: null plane");
    if ((((uintptr_t)out->rect) & 15) || (((uintptr_t)out->raster) & 63))
        return set_error(GS_ERR_INVALID, "gs_splats_from_2d: rect must be 16-byte and raster 64-byte aligned");
    hipLaunchKernelGGL(splats_from_2d_kernel, dim3(grid_for(n_splats, 256)), dim3(256), 0, (hipStream_t)stream, *g,
                       cams, (int)n_cams, n_splats, mean2d, conic, depth, valid, (RasterRec *)out->raster, out->depth,
                       (int4 *)out->rect, out->tiles_touched);
    return check_launch("gs_splats_from_2d");
}

extern "C" int gs_project(const gs_gaussians *g, const gs_camera *cams, int32_t n_cams, int64_t n_splats,
                          gs_splats *out, void *stream)
{
    clear_error();
    if (!g || !cams || !out || n_cams < 1 || n_splats < 0)
        return set_error(GS_ERR_INVALID, "gs_project: null argument or bad size");
    if (n_splats > out->capacity)
        return set_error(GS_ERR_INVALID, "gs_project: n_splats exceeds splat capacity");
    if (n_splats == 0) return GS_OK;
    if (!g->means || !g->quats || !g->scales || !g->colors || !g->opacities || g->n < 1 || !out->raster ||
        !out->depth || !out->rect || !out->tiles_touched)
        return set_error(GS_ERR_INVALID, "gs_project: null plane");
    if ((((uintptr_t)out->rec) & 15) || (((uintptr_t)out->rect) & 15) || (((uintptr_t)out->raster) & 63))
        return set_error(GS_ERR_INVALID, "gs_project: rec/rect must be 16-byte and raster 64-byte aligned");
    hipLaunchKernelGGL(project_kernel, dim3(grid_for(g->n, 256)), dim3(256), 0, (hipStream_t)stream, *g, cams,
                       (int)n_cams, n_splats, (float4 *)out->rec, (RasterRec *)out->raster, out->depth,
                       (int4 *)out->rect, out->tiles_touched);
    return check_launch("gs_project");
}
