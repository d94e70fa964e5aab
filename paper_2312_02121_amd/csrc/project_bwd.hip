// gs_project_bwd: gradients of the projection (Sec. 3.2, eqs. 22-28) and of the scale
// and rotation parameterisation (Sec. 3.2.1, eqs. 29-31). One thread per scene Gaussian,
// summing over the cameras that see it.
// The arithmetic is float64: dL/dSigma' = -Y dL/dY Y grows with the square of the conic,
// which is large for thin splats, and the chain that follows sums terms of both signs;
// in float32 that costs up to ~1e-3 of relative accuracy on single quaternion gradients.
// The kernel is HBM-bound (its float64 arithmetic, about half the float32 rate on gfx950,
// stays below the memory time). The conic Y in dL/dSigma' is re-derived here in float64 from Sigma' rather than read
// from the splat record: the record holds Y rounded to float32 for the compositing, and for a
// needle-like splat that rounding moves Y's small eigenvalue by up to ~1e-2 relative, which
// the product -Y dL/dY Y would carry into the gradient. The derivative of the inverse is
// taken at Sigma' itself.
//
// The mean route of eq. (23) is applied in its reduced form: with P of eq. (1), the
// product 1/2 P^T D^T dL/dmu' equals J^T dL/dmu' extended by 0, i.e.
//   dL/dt_x = f_x / t_z dmu'_x,  dL/dt_y = f_y / t_z dmu'_y,
//   dL/dt_z = -f_x t_x / t_z^2 dmu'_x - f_y t_y / t_z^2 dmu'_y.
#include "common.h"

namespace gsx {

// The gradients of one Gaussian through one camera's slot (float64).
struct GaussGrad {
    double dmu[3], ds[3], dq[4];
};

// One scene Gaussian as the backward reads it: mean, quaternion (normalised when asked), |q|
// and scale. R(q) and M = R(q) S are recomputed per camera rather than kept, which keeps the
// registers of the camera loop down.
struct GaussBwdIn {
    double mx, my, mz, qw, qx, qy, qz, qn, sv[3];
    bool normalize;   // q was normalised: dL/dq goes through q / |q|
};

__device__ inline GaussBwdIn load_gaussian_bwd(const gs_gaussians &g, int64_t i)
{
    const int64_t n = g.n;
    GaussBwdIn a;
    a.mx = g.means[i];
    a.my = g.means[n + i];
    a.mz = g.means[2 * n + i];
    a.qw = g.quats[i];
    a.qx = g.quats[n + i];
    a.qy = g.quats[2 * n + i];
    a.qz = g.quats[3 * n + i];
    a.qn = 1.0;   // |q| when normalised (same arithmetic as the projection)
    a.normalize = (g.flags & GS_NORMALIZE_QUATS) != 0;
    if (a.normalize) {
        a.qn = sqrt(a.qw * a.qw + a.qx * a.qx + a.qy * a.qy + a.qz * a.qz);
        a.qw = a.qw / a.qn;
        a.qx = a.qx / a.qn;
        a.qy = a.qy / a.qn;
        a.qz = a.qz / a.qn;
    }
    a.sv[0] = g.scales[i];
    a.sv[1] = g.scales[n + i];
    a.sv[2] = g.scales[2 * n + i];
    return a;
}

// Adds the gradients through camera c's slot p of Gaussian a (Sec. 3.2, 3.2.1) into acc and,
// with pose, writes that slot's camera-pose gradient (eq. 28 plus the R_cw term) into pose.
template <bool kPose>
__device__ inline void slot_backward(const gs_camera &cam, const GaussBwdIn &a, int64_t p, int64_t n_splats,
                                     const double *__restrict__ d_mean2d, const double *__restrict__ d_conic,
                                     GaussGrad &acc, float (&pose)[12])
{
    const double mx = a.mx, my = a.my, mz = a.mz;
    const double *sv = a.sv;
    const double qw = a.qw, qx = a.qx, qy = a.qy, qz = a.qz;
    const double Q[9] = {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy),
                         2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx),
                         2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)};
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b) M[3 * r + b] = Q[3 * r + b] * sv[b];
    double S[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            S[3 * r + b] = M[3 * r] * M[3 * b] + M[3 * r + 1] * M[3 * b + 1] + M[3 * r + 2] * M[3 * b + 2];
    const double R[9] = {cam.R[0], cam.R[1], cam.R[2], cam.R[3], cam.R[4], cam.R[5], cam.R[6], cam.R[7], cam.R[8]};
    const double fx = cam.fx, fy = cam.fy;

    // forward quantities
    const double tx = R[0] * mx + R[1] * my + R[2] * mz + cam.t[0];
    const double ty = R[3] * mx + R[4] * my + R[5] * mz + cam.t[1];
    const double tz = R[6] * mx + R[7] * my + R[8] * mz + cam.t[2];
    const double iz = 1.0 / tz, iz2 = iz * iz;
    const double J00 = fx * iz, J02 = -fx * tx * iz2, J11 = fy * iz, J12 = -fy * ty * iz2;
    double T[6];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T[j] = J00 * R[j] + J02 * R[6 + j];
        T[3 + j] = J11 * R[3 + j] + J12 * R[6 + j];
    }
    // Sigma' = T Sigma T^T (eq. 4) and Y = Sigma'^-1, in float64
    double TS[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            TS[3 * r + b] = T[3 * r] * S[b] + T[3 * r + 1] * S[3 + b] + T[3 * r + 2] * S[6 + b];
    const double C00 = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2];
    const double C01 = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
    const double C11 = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5];
    const double det = C00 * C11 - C01 * C01;
    const double y00 = C11 / det, y01 = -C01 / det, y11 = C00 / det;

    // dL/dSigma' = -Y dL/dY Y (Sec. 3.1), Y symmetric
    const double g00 = d_conic[p], g01 = d_conic[n_splats + p], g11 = d_conic[2 * n_splats + p];
    const double a00 = y00 * g00 + y01 * g01, a01 = y00 * g01 + y01 * g11;   // Y G
    const double a10 = y01 * g00 + y11 * g01, a11 = y01 * g01 + y11 * g11;
    const double G00 = -(a00 * y00 + a01 * y01), G01 = -(a00 * y01 + a01 * y11);
    const double G10 = -(a10 * y00 + a11 * y01), G11 = -(a10 * y01 + a11 * y11);

    // mean route (eq. 23 reduced)
    const double dmx = d_mean2d[p], dmy = d_mean2d[n_splats + p];
    double dtx = J00 * dmx, dty = J11 * dmy, dtz = J02 * dmx + J12 * dmy;

    // covariance route: dL/dT = G T Sigma + G^T T Sigma (eq. 25), dL/dJ = dL/dT R_cw^T
    double dT[6];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        dT[b] = (G00 + G00) * TS[b] + (G01 + G10) * TS[3 + b];
        dT[3 + b] = (G10 + G01) * TS[b] + (G11 + G11) * TS[3 + b];
    }
    double dJ[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            dJ[3 * r + a] = dT[3 * r] * R[3 * a] + dT[3 * r + 1] * R[3 * a + 1] + dT[3 * r + 2] * R[3 * a + 2];
    // dJ/dt (Sec. 3.2)
    const double iz3 = iz2 * iz;
    dtx += dJ[2] * (-fx * iz2);
    dty += dJ[5] * (-fy * iz2);
    dtz += dJ[0] * (-fx * iz2) + dJ[2] * (2.0 * fx * tx * iz3) + dJ[4] * (-fy * iz2) + dJ[5] * (2.0 * fy * ty * iz3);

    // eq. (28): dL/dmu = R_cw^T dL/dt
    const double dmu0 = R[0] * dtx + R[3] * dty + R[6] * dtz;
    const double dmu1 = R[1] * dtx + R[4] * dty + R[7] * dtz;
    const double dmu2 = R[2] * dtx + R[5] * dty + R[8] * dtz;

    // eq. (24): dL/dSigma = T^T G T
    double GT[6];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        GT[b] = G00 * T[b] + G01 * T[3 + b];
        GT[3 + b] = G10 * T[b] + G11 * T[3 + b];
    }
    double dS[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) dS[3 * a + b] = T[a] * GT[b] + T[3 + a] * GT[3 + b];
    // eq. (29): dL/dM = (dL/dSigma + dL/dSigma^T) M
    double dM[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            dM[3 * a + b] = (dS[3 * a] + dS[a]) * M[b] + (dS[3 * a + 1] + dS[3 + a]) * M[3 + b] +
                            (dS[3 * a + 2] + dS[6 + a]) * M[6 + b];
    // eq. (30): dL/dR = dL/dM S^T, dL/dS = R^T dL/dM; eq. (31) keeps its diagonal
    double dR[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) dR[3 * a + b] = dM[3 * a + b] * sv[b];
    double ds[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) ds[b] = Q[b] * dM[b] + Q[3 + b] * dM[3 + b] + Q[6 + b] * dM[6 + b];
    // dR/dq (Sec. 3.2.1), q = (w, x, y, z)
    double dqw = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
    double dqx = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - qw * dR[5] + qz * dR[6] +
                        qw * dR[7] - 2.0 * qx * dR[8]);
    double dqy = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] - qw * dR[6] +
                        qz * dR[7] - 2.0 * qy * dR[8]);
    double dqz = 2.0 * (-2.0 * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] - 2.0 * qz * dR[4] +
                        qy * dR[5] + qx * dR[6] + qy * dR[7]);
    if (a.normalize) {
        // through q^ = q / |q|: d q^ / d q = (I - q^ q^T) / |q|
        const double dot = qw * dqw + qx * dqx + qy * dqy + qz * dqz;
        dqw = (dqw - qw * dot) / a.qn;
        dqx = (dqx - qx * dot) / a.qn;
        dqy = (dqy - qy * dot) / a.qn;
        dqz = (dqz - qz * dot) / a.qn;
    }

    acc.dmu[0] += dmu0;
    acc.dmu[1] += dmu1;
    acc.dmu[2] += dmu2;
    acc.ds[0] += ds[0];
    acc.ds[1] += ds[1];
    acc.ds[2] += ds[2];
    acc.dq[0] += dqw;
    acc.dq[1] += dqx;
    acc.dq[2] += dqy;
    acc.dq[3] += dqz;

    if (kPose) {
        // eq. (28): dL/dT_cw = dL/dt [mu; 1]^T, plus J^T dL/dT for R_cw entering T = J R_cw
        const double dt[3] = {dtx, dty, dtz}, mu[3] = {mx, my, mz};
        const double JtdT[9] = {J00 * dT[0], J00 * dT[1], J00 * dT[2],
                               J11 * dT[3], J11 * dT[4], J11 * dT[5],
                               J02 * dT[0] + J12 * dT[3], J02 * dT[1] + J12 * dT[4], J02 * dT[2] + J12 * dT[5]};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int b = 0; b < 3; ++b) pose[4 * r + b] = (float)(dt[r] * mu[b] + JtdT[3 * r + b]);
            pose[4 * r + 3] = (float)dt[r];
        }
    }
}

// Gaussian-major: one thread per scene Gaussian. It walks the cameras that view its scene and,
// for each camera's slot where the splat was listed (tiles_touched > 0), computes the
// gradients through that slot in float64; their float32 sum over the cameras goes into the
// scene gradients with one plain read-modify-write per value (no other thread owns the
// Gaussian, so no atomics). The Gaussian's parameters are re-read per camera (cache hits)
// rather than kept in registers across the loop. The camera-pose gradient of each camera
// is summed over the wave and added with one atomic per value and wave.
template <bool kPose>
__global__ __launch_bounds__(256) void project_bwd_kernel(gs_gaussians g, const gs_camera *__restrict__ cams, int n_cams,
                                                          const int32_t *__restrict__ tiles, int64_t n_splats,
                                                          const double *__restrict__ d_mean2d,
                                                          const double *__restrict__ d_conic, float *__restrict__ d_means,
                                                          float *__restrict__ d_scales, float *__restrict__ d_quats,
                                                          float *__restrict__ d_pose)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = g.n;
    const bool in_range = i < n;
    // the Gaussian's sums over cameras, float32 like the scene gradients they are added to
    float sum[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) sum[q] = 0.f;
    bool any = false;
#pragma unroll 1
    for (int c = 0; c < n_cams; ++c) {
        const gs_camera &cam = cams[c];
        const int64_t k = i - cam.gauss_offset;
        const int64_t p = cam.proj_offset + k;
        const bool live = in_range && k >= 0 && k < cam.gauss_count && p < n_splats && tiles[p] > 0;
        float pose[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) pose[q] = 0.f;
        if (live) {
            const GaussBwdIn a = load_gaussian_bwd(g, i);
            GaussGrad acc;
#pragma unroll
            for (int q = 0; q < 3; ++q) acc.dmu[q] = acc.ds[q] = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc.dq[q] = 0.0;
            slot_backward<kPose>(cam, a, p, n_splats, d_mean2d, d_conic, acc, pose);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                sum[q] += (float)acc.dmu[q];
                sum[3 + q] += (float)acc.ds[q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[6 + q] += (float)acc.dq[q];
            any = true;
        }
        if (kPose && __ballot(live) != 0) {
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const float tot = wave_sum_to_lane63(pose[q]);
                if ((threadIdx.x & (kWave - 1)) == kWave - 1) atomic_add_f32(&d_pose[12 * c + q], tot);
            }
        }
    }
    if (any) {
        d_means[i] += sum[0];
        d_means[n + i] += sum[1];
        d_means[2 * n + i] += sum[2];
        d_scales[i] += sum[3];
        d_scales[n + i] += sum[4];
        d_scales[2 * n + i] += sum[5];
        d_quats[i] += sum[6];
        d_quats[n + i] += sum[7];
        d_quats[2 * n + i] += sum[8];
        d_quats[3 * n + i] += sum[9];
    }
}

}  // namespace gsx

using namespace gsx;

extern "C" int gs_project_bwd(const gs_gaussians *g, const gs_camera *cams, int32_t n_cams, const gs_splats *s,
                              int64_t n_splats, const double *dL_dmean2d, const double *dL_dconic, float *dL_dmeans,
                              float *dL_dscales, float *dL_dquats, float *dL_dcampose, void *stream)
{
    clear_error();
    if (!g || !cams || !s || n_cams < 1 || n_splats < 0 || n_splats > s->capacity || !dL_dmean2d || !dL_dconic ||
        !dL_dmeans || !dL_dscales || !dL_dquats || !s->tiles_touched)
        return set_error(GS_ERR_INVALID, "gs_project_bwd: null argument or bad size");
    if (!g->means || !g->quats || !g->scales || g->n < 1)
        return set_error(GS_ERR_INVALID, "gs_project_bwd: null Gaussian plane");
    if (n_splats == 0) return GS_OK;
    if (dL_dcampose)
        hipLaunchKernelGGL(project_bwd_kernel<true>, dim3(grid_for(g->n, 256)), dim3(256), 0, (hipStream_t)stream, *g,
                           cams, (int)n_cams, s->tiles_touched, n_splats, dL_dmean2d, dL_dconic, dL_dmeans, dL_dscales,
                           dL_dquats, dL_dcampose);
    else
        hipLaunchKernelGGL(project_bwd_kernel<false>, dim3(grid_for(g->n, 256)), dim3(256), 0, (hipStream_t)stream, *g,
                           cams, (int)n_cams, s->tiles_touched, n_splats, dL_dmean2d, dL_dconic, dL_dmeans, dL_dscales,
                           dL_dquats, dL_dcampose);
    return check_launch("gs_project_bwd");
}
