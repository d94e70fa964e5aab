/*
 * gs_oracle.c -- plain CPU FP64 oracle for the differentiable tile rasterizer of
 * 3D Gaussians (gsplat mathematical supplement, arXiv 2312.02121).
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's CPU
 * baseline load this library; the product path never does. It shares no code,
 * header, table or helper with the HIP library.
 *
 * Everything is computed in double precision from the paper's definitions, in
 * the paper's order:
 *   projection              Sec. 2.1, eqs. (1)-(6)
 *   tile binning and sort   Sec. 2.2 (16x16 tiles, 3-sigma box, per-tile depth order)
 *   compositing             Sec. 2.2, eq. (7) and the alpha/sigma definitions after it
 *   compositing gradients   Sec. 3.1, eqs. (16)-(21)
 *   projection gradients    Sec. 3.2, eqs. (22)-(28); scale/rotation Sec. 3.2.1, eqs. (29)-(31)
 *
 * Readings of places where the paper is silent or misprinted (each is pinned by a
 * test; the `errata` bits reproduce the printed form so that the test can show the
 * pin catches it):
 *   - eq. (5): the printed R11 = 1 - 2(x^2 - z^2) is not a rotation; we use
 *     1 - 2(x^2 + z^2), the only form consistent with dR/dz in Sec. 3.2.1.
 *   - quaternions are stored (w, x, y, z), the order of Sec. 3.2.1, and are not
 *     renormalised (the paper's R(q) assumes a unit q). As an option
 *     (normalize_quats), q is replaced by q / |q| before R(q), and dL/dq becomes
 *     (dL/dq^ - q^ (q^ . dL/dq^)) / |q| with q^ = q / |q|.
 *   - Delta = mu' - p (pixel centre p), the sign for which dsigma/dmu' = Y Delta.
 *   - eq. (23): the second row uses h, and t means t' there.
 *   - near/far cull: keep only near < t_z < far, and t_z > 0 (depth keys are float bits).
 *   - 3-sigma box: tight axis-aligned half extents 3 sqrt(Sigma'_00), 3 sqrt(Sigma'_11).
 *     As an option (box_lambda_max), a square of half extent 3 sqrt(lambda_max) with
 *     lambda_max = (a + c) / 2 + sqrt(((a - c) / 2)^2 + b^2), Sigma' = (a, b; b, c):
 *     the largest eigenvalue, so the square contains the tight box.
 *   - tile k spans pixel coordinates [16k, 16k+16); pixel (row i, col j) has centre
 *     (j + 1/2, i + 1/2).
 *   - alpha = min(alpha_max, o exp(-sigma)); entries with alpha < alpha_min are
 *     skipped; compositing stops before the first entry whose T (1 - alpha) would
 *     fall below T_min. Literal mode is alpha_min = 0, alpha_max = 1, T_min = 0.
 *   - symmetric-matrix gradients are full-matrix gradients; the off-diagonal of a
 *     stored 2x2 conic gradient is the (0,1) entry, not doubled.
 *   - camera-pose gradient: eq. (28) accounts for T_cw through t only; R_cw also
 *     enters Sigma' through T = J R_cw, and that term is added.
 *   - background: the image formation of Sec. 2.2 has none (a background of zero).
 *     As an option, a colour bg is seen through what is left of the pixel:
 *     C = sum_n c_n alpha_n T_n + T_final bg. In the backward bg acts as one more
 *     colour behind the last composited entry, with weight T_final, so it enters
 *     S(n) of eq. (18) for every entry.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math -fopenmp
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16

enum {
    ORC_ERRATA_R11 = 1,      /* printed sign of R11 in eq. (5) */
    ORC_ERRATA_EQ23_W = 2,   /* printed w (instead of h) in the second row of eq. (23) */
    ORC_ERRATA_DELTA = 4,    /* Delta = p - mu' together with dsigma/dmu' = Y Delta */
    ORC_ERRATA_EQ28_ONLY = 8 /* camera-pose gradient through t alone, as eq. (28) prints it */
};

typedef struct {
    double R[9];         /* R_cw, row-major */
    double t[3];         /* t_cw */
    double fx, fy, cx, cy;
    int64_t W, H;
    double near_plane, far_plane;
} orc_camera;

typedef struct {
    double alpha_min, alpha_max, T_min;
    /* Near-tie flags. A float32 implementation takes the skip, termination and clamp
     * decisions on rounded values; a pixel whose exact decision quantity lies within the
     * implementation's error bound of a threshold may go either way there, and is flagged.
     * The bounds describe that implementation and are passed in by the caller: */
    double margin_alpha;   /* relative error bound of its alpha: flag a pixel if
                              |alpha - alpha_min| <= margin_alpha * alpha_min */
    double margin_T;       /* ... or |T (1 - alpha) - T_min| <= e_T * max(T (1 - alpha), T_min), with
                              e_T = margin_T + sum over the factors of T (1 - alpha) so far of
                                    round_T + (alpha clamped ? 0 : margin_alpha * alpha / (1 - alpha)):
                              a first-order bound on the relative error of its product T,
                              each factor carrying one rounding of the update (round_T) and the
                              error of its alpha, which a clamped alpha (exactly alpha_max)
                              does not have (e_T is taken as 0 when margin_T is 0) */
    double margin_clamp;   /* ... or |o exp(-sigma) - alpha_max| <= margin_clamp */
    int32_t round_interface; /* round mu', Y, depth to float32 where the HIP path stores them */
    int32_t errata;
    int32_t n_threads;     /* <= 0: OpenMP default */
    int32_t normalize_quats; /* 1: R(q / |q|) (an option; the paper uses q as given) */
    double background[3];  /* bg, zero for the paper's image formation */
    int32_t box_lambda_max;  /* 1: square 3-sigma box from the largest eigenvalue of Sigma' */
    int32_t pad2;
    double round_T;        /* relative rounding bound of one float32 update of T (see margin_T) */
} orc_params;

/* ------------------------------------------------------------------ small linear algebra */

/* C[m x n] = A[m x k] B[k x n], all row-major; sums run left to right. */
static void mm(const double *A, const double *B, double *C, int m, int k, int n)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int l = 0; l < k; ++l)
                acc += A[i * k + l] * B[l * n + j];
            C[i * n + j] = acc;
        }
}

static void tr(const double *A, double *At, int m, int n)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            At[j * m + i] = A[i * n + j];
}

/* Frobenius inner product <X, Y> (Sec. 3) */
static double frob(const double *X, const double *Y, int count)
{
    double acc = 0.0;
    for (int i = 0; i < count; ++i)
        acc += X[i] * Y[i];
    return acc;
}

static int all_finite(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i]))
            return 0;
    return 1;
}

static double round_f32(double x) { return (double)(float)x; }

/* ---------------------------------------------------------------------- projection */

/* eq. (5), q = (w, x, y, z). */
void orc_quat_to_rot(const double *q, int errata, double *R)
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = (errata & ORC_ERRATA_R11) ? 1.0 - 2.0 * (x * x - z * z) : 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* eq. (6): Sigma = R S S^T R^T with S = diag(s); M = R S so Sigma = M M^T. */
void orc_cov3d(const double *q, const double *s, int errata, double *R, double *M, double *Sigma)
{
    double S[9] = {s[0], 0.0, 0.0, 0.0, s[1], 0.0, 0.0, 0.0, s[2]};
    double Mt[9];
    orc_quat_to_rot(q, errata, R);
    mm(R, S, M, 3, 3, 3);
    tr(M, Mt, 3, 3);
    mm(M, Mt, Sigma, 3, 3, 3);
}

/* eq. (1): the projection matrix P. */
static void proj_matrix(const orc_camera *c, double *P)
{
    const double w = (double)c->W, h = (double)c->H, n = c->near_plane, f = c->far_plane;
    memset(P, 0, 16 * sizeof(double));
    P[0] = 2.0 * c->fx / w;
    P[5] = 2.0 * c->fy / h;
    P[10] = (f + n) / (f - n);
    P[11] = -2.0 * f * n / (f - n);
    P[14] = 1.0;
}

typedef struct {
    double mu[3], q[4], s[3];
    double qn;                  /* |q| when q was normalised, else 1 */
    double R[9], M[9], Sigma[9];
    double t[4], tp[4];         /* t = T_cw [mu; 1], t' = P t (eq. 2) */
    double J[6], T[6];          /* eq. (3) and T = J R_cw */
    double cov2d[4];            /* Sigma' (eq. 4), 2x2 row-major */
    double det, Y[4];           /* Y = Sigma'^{-1} */
    double mean2d[2];           /* mu' (eq. 2) */
    double depth;
    int64_t rect[4];            /* tile x0, y0, x1, y1 inclusive */
    int64_t tiles;
} orc_proj;

/* Projects one Gaussian; returns 1 if it survives culling. */
static int project_one(const orc_camera *cam, const orc_params *prm, orc_proj *g)
{
    g->tiles = 0;
    g->rect[0] = g->rect[1] = g->rect[2] = g->rect[3] = 0;
    g->qn = 1.0;
    if (prm->normalize_quats) {
        /* a zero or non-finite q gives a non-finite q^, which is culled below */
        const double qn = sqrt(g->q[0] * g->q[0] + g->q[1] * g->q[1] + g->q[2] * g->q[2] + g->q[3] * g->q[3]);
        for (int a = 0; a < 4; ++a) g->q[a] = g->q[a] / qn;
        g->qn = qn;
    }
    if (!all_finite(g->mu, 3) || !all_finite(g->q, 4) || !all_finite(g->s, 3))
        return 0;
    orc_cov3d(g->q, g->s, prm->errata, g->R, g->M, g->Sigma);

    /* t = T_cw [mu; 1] */
    double Tcw[16] = {cam->R[0], cam->R[1], cam->R[2], cam->t[0],
                      cam->R[3], cam->R[4], cam->R[5], cam->t[1],
                      cam->R[6], cam->R[7], cam->R[8], cam->t[2],
                      0.0, 0.0, 0.0, 1.0};
    double hom[4] = {g->mu[0], g->mu[1], g->mu[2], 1.0};
    mm(Tcw, hom, g->t, 4, 4, 1);
    if (!all_finite(g->t, 3))
        return 0;
    const double tx = g->t[0], ty = g->t[1], tz = g->t[2];
    /* keep near < t_z < far; t_z <= 0 is culled whatever the near plane: the depth order of
     * Sec. 2.2 is taken on the float32 bits of t_z, which order only positive values */
    if (!(tz > cam->near_plane) || !(tz > 0.0) || !(tz < cam->far_plane))
        return 0;

    /* t' = P t and mu' (eq. 2) */
    double P[16];
    proj_matrix(cam, P);
    mm(P, g->t, g->tp, 4, 4, 1);
    const double w = (double)cam->W, h = (double)cam->H;
    g->mean2d[0] = (w * g->tp[0] / g->tp[3] + 1.0) / 2.0 + cam->cx;
    g->mean2d[1] = (h * g->tp[1] / g->tp[3] + 1.0) / 2.0 + cam->cy;
    g->depth = tz;

    /* eq. (3) */
    g->J[0] = cam->fx / tz;  g->J[1] = 0.0;  g->J[2] = -(cam->fx * tx) / (tz * tz);
    g->J[3] = 0.0;  g->J[4] = cam->fy / tz;  g->J[5] = -(cam->fy * ty) / (tz * tz);

    /* eq. (4): Sigma' = J R_cw Sigma R_cw^T J^T = T Sigma T^T with T = J R_cw */
    double U[6], Tt[6];
    mm(g->J, cam->R, g->T, 2, 3, 3);
    mm(g->T, g->Sigma, U, 2, 3, 3);
    tr(g->T, Tt, 2, 3);
    mm(U, Tt, g->cov2d, 2, 3, 2);
    /* the stored Sigma' is symmetric by construction: its (1,0) entry is taken as (0,1) */
    g->cov2d[2] = g->cov2d[1];
    g->det = g->cov2d[0] * g->cov2d[3] - g->cov2d[1] * g->cov2d[1];
    if (!all_finite(g->cov2d, 4) || !(g->det > 0.0) || !(g->cov2d[0] > 0.0) || !(g->cov2d[3] > 0.0))
        return 0;
    g->Y[0] = g->cov2d[3] / g->det;
    g->Y[1] = -g->cov2d[1] / g->det;
    g->Y[2] = g->Y[1];
    g->Y[3] = g->cov2d[0] / g->det;
    if (!all_finite(g->mean2d, 2) || !all_finite(g->Y, 4))
        return 0;

    /* Sec. 2.2: axis-aligned box of the 3-sigma ellipse, intersected with the tile grid */
    double ex = 3.0 * sqrt(g->cov2d[0]);
    double ey = 3.0 * sqrt(g->cov2d[3]);
    if (prm->box_lambda_max) {
        const double a = g->cov2d[0], b = g->cov2d[1], c = g->cov2d[3];
        const double h = (a - c) / 2.0;
        const double lmax = (a + c) / 2.0 + sqrt(h * h + b * b);
        ex = ey = 3.0 * sqrt(lmax);
    }
    const double TX = (double)((cam->W + ORC_TILE - 1) / ORC_TILE);
    const double TY = (double)((cam->H + ORC_TILE - 1) / ORC_TILE);
    double x0 = floor((g->mean2d[0] - ex) / ORC_TILE);
    double x1 = floor((g->mean2d[0] + ex) / ORC_TILE);
    double y0 = floor((g->mean2d[1] - ey) / ORC_TILE);
    double y1 = floor((g->mean2d[1] + ey) / ORC_TILE);
    if (!(x1 >= 0.0) || !(y1 >= 0.0) || !(x0 <= TX - 1.0) || !(y0 <= TY - 1.0))
        return 0;
    if (x0 < 0.0) x0 = 0.0;
    if (y0 < 0.0) y0 = 0.0;
    if (x1 > TX - 1.0) x1 = TX - 1.0;
    if (y1 > TY - 1.0) y1 = TY - 1.0;
    g->rect[0] = (int64_t)x0;
    g->rect[1] = (int64_t)y0;
    g->rect[2] = (int64_t)x1;
    g->rect[3] = (int64_t)y1;
    g->tiles = (g->rect[2] - g->rect[0] + 1) * (g->rect[3] - g->rect[1] + 1);
    return 1;
}

static void load_gaussian(int64_t N, int64_t i, const double *means, const double *quats,
                          const double *scales, orc_proj *g)
{
    for (int a = 0; a < 3; ++a) g->mu[a] = means[a * N + i];
    for (int a = 0; a < 4; ++a) g->q[a] = quats[a * N + i];
    for (int a = 0; a < 3; ++a) g->s[a] = scales[a * N + i];
}

static void set_threads(const orc_params *prm)
{
#ifdef _OPENMP
    if (prm && prm->n_threads > 0)
        omp_set_num_threads(prm->n_threads);
#else
    (void)prm;
#endif
}

/*
 * Projection of N Gaussians through one camera (Sec. 2.1 and the box of Sec. 2.2).
 * Outputs: mean2d [2][N], conic [3][N] = (Y00, Y01, Y11), depth [N], rect [4][N],
 * tiles_touched [N]. Culled Gaussians get tiles_touched = 0 and zero outputs.
 * Returns the number of visible Gaussians.
 */
int64_t orc_project(int64_t N, const double *means, const double *quats, const double *scales,
                    const orc_camera *cam, const orc_params *prm,
                    double *mean2d, double *conic, double *depth, int32_t *rect, int32_t *tiles)
{
    int64_t visible = 0;
    set_threads(prm);
#pragma omp parallel for reduction(+ : visible) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        orc_proj g;
        load_gaussian(N, i, means, quats, scales, &g);
        int ok = project_one(cam, prm, &g);
        if (!ok) {
            mean2d[i] = mean2d[N + i] = 0.0;
            conic[i] = conic[N + i] = conic[2 * N + i] = 0.0;
            depth[i] = 0.0;
            for (int a = 0; a < 4; ++a) rect[a * N + i] = 0;
            tiles[i] = 0;
            continue;
        }
        visible += 1;
        double m0 = g.mean2d[0], m1 = g.mean2d[1], y0 = g.Y[0], y1 = g.Y[1], y2 = g.Y[3], d = g.depth;
        if (prm->round_interface) {
            m0 = round_f32(m0); m1 = round_f32(m1);
            y0 = round_f32(y0); y1 = round_f32(y1); y2 = round_f32(y2);
            d = round_f32(d);
        }
        mean2d[i] = m0; mean2d[N + i] = m1;
        conic[i] = y0; conic[N + i] = y1; conic[2 * N + i] = y2;
        depth[i] = d;
        for (int a = 0; a < 4; ++a) rect[a * N + i] = (int32_t)g.rect[a];
        tiles[i] = (int32_t)g.tiles;
    }
    return visible;
}

/* ------------------------------------------------------------------ binning and sorting */

typedef struct { uint64_t key; int32_t id; } orc_entry;

static int cmp_entry(const void *a, const void *b)
{
    const orc_entry *x = (const orc_entry *)a, *y = (const orc_entry *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

static uint64_t depth_bits(double depth)
{
    float f = (float)depth;
    uint32_t u;
    memcpy(&u, &f, 4);
    return (uint64_t)u;
}

/*
 * Sec. 2.2: each visible Gaussian joins every tile its box intersects; each tile's
 * list is ordered by depth. Keys are (global tile << 32) | float32 depth bits, ties
 * broken by the Gaussian index. K must be sum(tiles_touched). tile_offset shifts the
 * camera's tile ids into a shared key space.
 */
void orc_bin_and_sort(int64_t N, const int32_t *rect, const double *depth, const int32_t *tiles,
                      int64_t tiles_x, int64_t tile_offset, int64_t K, uint64_t *keys, int32_t *ids)
{
    orc_entry *e = (orc_entry *)malloc((size_t)(K > 0 ? K : 1) * sizeof(orc_entry));
    int64_t k = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (tiles[i] <= 0) continue;
        for (int64_t ty = rect[N + i]; ty <= rect[3 * N + i]; ++ty)
            for (int64_t tx = rect[i]; tx <= rect[2 * N + i]; ++tx) {
                uint64_t tile = (uint64_t)(tile_offset + ty * tiles_x + tx);
                e[k].key = (tile << 32) | depth_bits(depth[i]);
                e[k].id = (int32_t)i;
                ++k;
            }
    }
    qsort(e, (size_t)k, sizeof(orc_entry), cmp_entry);
    for (int64_t j = 0; j < k; ++j) {
        keys[j] = e[j].key;
        ids[j] = e[j].id;
    }
    free(e);
}

/* [start, end) of each tile's run in the sorted list; empty tiles get (0, 0). */
void orc_tile_ranges(int64_t K, const uint64_t *keys, int64_t n_tiles, int64_t tile_offset, int64_t *ranges)
{
    for (int64_t t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
    for (int64_t k = 0; k < K; ++k) {
        int64_t t = (int64_t)(keys[k] >> 32) - tile_offset;
        if (t < 0 || t >= n_tiles) continue;
        if (k == 0 || (keys[k - 1] >> 32) != (keys[k] >> 32)) ranges[2 * t] = k;
        if (k == K - 1 || (keys[k + 1] >> 32) != (keys[k] >> 32)) ranges[2 * t + 1] = k + 1;
    }
}

/* ------------------------------------------------------------------------ compositing */

/* sigma_n = 1/2 Delta^T Y Delta with Delta = mu' - p (text after eq. 7) */
static double sigma_of(const double *Y3, double dx, double dy)
{
    return 0.5 * (dx * (Y3[0] * dx + Y3[1] * dy) + dy * (Y3[1] * dx + Y3[2] * dy));
}

/* eq. (7) for one pixel with centre (px, py) over the list entries [start, end): outputs
 * the colour (background seen through T_final), T_final, last (one past the list position
 * of the last composited entry), visited (entries whose alpha was evaluated, including a
 * terminating one) and flags (near-tie decisions: 1 skip threshold, 2 termination,
 * 4 clamp). */
static void composite_pixel(int64_t N, const double *mean2d, const double *conic, const double *colors,
                            const double *opac, const int32_t *ids, int64_t start, int64_t end,
                            double px, double py, const orc_params *prm,
                            double *rgb, double *T_out, int32_t *last, int32_t *visited, int32_t *flags)
{
    double T = 1.0, c0 = 0.0, c1 = 0.0, c2 = 0.0, eT = prm->margin_T;
    int32_t nlast = 0, nvis = 0, fl = 0;
    for (int64_t k = start; k < end; ++k) {
        const int32_t g = ids[k];
        const double Y3[3] = {conic[g], conic[N + g], conic[2 * N + g]};
        const double dx = mean2d[g] - px, dy = mean2d[N + g] - py;
        const double a_raw = opac[g] * exp(-sigma_of(Y3, dx, dy));
        ++nvis;
        if (fabs(a_raw - prm->alpha_max) <= prm->margin_clamp) fl |= 4;
        const double alpha = a_raw < prm->alpha_max ? a_raw : prm->alpha_max;
        /* with alpha_min = 0 (literal mode) there is no skip decision to flag */
        if (prm->alpha_min > 0.0 && fabs(alpha - prm->alpha_min) <= prm->margin_alpha * prm->alpha_min) fl |= 1;
        if (alpha < prm->alpha_min) continue;
        const double Tn = T * (1.0 - alpha);
        const double eTn = prm->margin_T > 0.0
            ? eT + prm->round_T + (a_raw >= prm->alpha_max ? 0.0 : prm->margin_alpha * alpha / (1.0 - alpha))
            : 0.0;
        /* with T_min = 0 (literal mode) there is no termination decision to flag */
        if (prm->T_min > 0.0 && fabs(Tn - prm->T_min) <= eTn * (Tn > prm->T_min ? Tn : prm->T_min)) fl |= 2;
        if (Tn < prm->T_min) break;
        eT = eTn;
        c0 += colors[g] * alpha * T;
        c1 += colors[N + g] * alpha * T;
        c2 += colors[2 * N + g] * alpha * T;
        T = Tn;
        nlast = (int32_t)(k - start + 1);
    }
    rgb[0] = c0 + T * prm->background[0];
    rgb[1] = c1 + T * prm->background[1];
    rgb[2] = c2 + T * prm->background[2];
    *T_out = T;
    *last = nlast;
    *visited = nvis;
    *flags = fl;
}

/*
 * eq. (7) per pixel over its tile's depth-ordered list.
 * colors [3][N], opac [N] are per projected Gaussian. Outputs C [3][W*H], T_final, last,
 * visited and flags per pixel (see composite_pixel; visited and flags may be NULL).
 */
void orc_rasterize_fwd(int64_t N, const double *mean2d, const double *conic, const double *colors,
                       const double *opac, const int32_t *ids, const int64_t *ranges,
                       int64_t W, int64_t H, const orc_params *prm,
                       double *C, double *T_final, int32_t *last, int32_t *visited, int32_t *flags)
{
    const int64_t TX = (W + ORC_TILE - 1) / ORC_TILE;
    const int64_t HW = W * H;
    set_threads(prm);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < H; ++i) {
        for (int64_t j = 0; j < W; ++j) {
            const int64_t pix = i * W + j;
            const int64_t tile = (i / ORC_TILE) * TX + (j / ORC_TILE);
            double rgb[3];
            int32_t nvis, fl;
            composite_pixel(N, mean2d, conic, colors, opac, ids, ranges[2 * tile], ranges[2 * tile + 1],
                            (double)j + 0.5, (double)i + 0.5, prm, rgb, &T_final[pix], &last[pix], &nvis, &fl);
            C[pix] = rgb[0];
            C[HW + pix] = rgb[1];
            C[2 * HW + pix] = rgb[2];
            if (visited) visited[pix] = nvis;
            if (flags) flags[pix] = fl;
        }
    }
}

/*
 * eq. (7) on a subset of tiles only: the n_sel tiles sel[] (tile indices of a W x H
 * camera), each with its depth-ordered list ids[ranges[2t] .. ranges[2t+1]). Pixels of
 * tile sel[s] are written at [s][row][col] of a 16 x 16 block (rows and columns past the
 * image edge are left untouched): C [3][n_sel][256], T_final, last, flags [n_sel][256]
 * (each may be NULL).
 * Returns sum over the written pixels and channels of (C - target)^2, target [3][W*H]
 * (NULL: no loss). The arithmetic per pixel is composite_pixel, as in orc_rasterize_fwd.
 */
double orc_rasterize_tiles(int64_t N, const double *mean2d, const double *conic, const double *colors,
                           const double *opac, const int32_t *ids, const int64_t *ranges,
                           int64_t W, int64_t H, const orc_params *prm, int64_t n_sel, const int64_t *sel,
                           const double *target, double *C, double *T_final, int32_t *last, int32_t *flags)
{
    const int64_t TX = (W + ORC_TILE - 1) / ORC_TILE;
    const int64_t HW = W * H, B = ORC_TILE * ORC_TILE;
    double loss = 0.0;
    set_threads(prm);
    /* per-tile partial sums, added in tile order, so the loss does not depend on threads */
    double *part = (double *)calloc((size_t)(n_sel > 0 ? n_sel : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sel; ++s) {
        const int64_t t = sel[s], ty = t / TX, tx = t % TX;
        double acc = 0.0;
        for (int64_t r = 0; r < ORC_TILE; ++r)
            for (int64_t c = 0; c < ORC_TILE; ++c) {
                const int64_t i = ty * ORC_TILE + r, j = tx * ORC_TILE + c;
                if (i >= H || j >= W) continue;
                double rgb[3], T;
                int32_t nl, nv, fl;
                composite_pixel(N, mean2d, conic, colors, opac, ids, ranges[2 * t], ranges[2 * t + 1],
                                (double)j + 0.5, (double)i + 0.5, prm, rgb, &T, &nl, &nv, &fl);
                const int64_t o = s * B + r * ORC_TILE + c;
                if (C) {
                    C[o] = rgb[0];
                    C[n_sel * B + o] = rgb[1];
                    C[2 * n_sel * B + o] = rgb[2];
                }
                if (T_final) T_final[o] = T;
                if (last) last[o] = nl;
                if (flags) flags[o] = fl;
                if (target) {
                    const int64_t pix = i * W + j;
                    for (int ch = 0; ch < 3; ++ch) {
                        const double d = rgb[ch] - target[ch * HW + pix];
                        acc += d * d;
                    }
                }
            }
        part[s] = acc;
    }
    for (int64_t s = 0; s < n_sel; ++s) loss += part[s];
    free(part);
    return loss;
}

/*
 * Sec. 3.1 for one pixel, walking back from its last composited entry.
 * form 0: T recovered by division from T_final (eq. 17), S by the backward
 *         recurrence, summed over channels against dL/dC.
 * form 1: T_n as the forward product and S_n(k) as the explicit sum over m > n,
 *         per channel (eq. 18 as printed); quadratic in the list length.
 * Per-entry gradients are added into g9[k - start][0..8] =
 *   (dmu'_x, dmu'_y, dY00, dY01, dY11, dc0, dc1, dc2, do).
 */
static void pixel_backward(int64_t N, const double *mean2d, const double *conic, const double *colors,
                           const double *opac, const int32_t *ids, int64_t start, int64_t nlast,
                           double px, double py, const double *g, double T_fin, const orc_params *prm,
                           int form, double *g9)
{
    const int delta_flip = (prm->errata & ORC_ERRATA_DELTA) != 0;
    const double *bg = prm->background;
    if (form == 0) {
        /* the background is the colour behind the last entry, seen with weight T_final */
        double T = T_fin, gS = (g[0] * bg[0] + g[1] * bg[1] + g[2] * bg[2]) * T_fin;
        for (int64_t k = start + nlast - 1; k >= start; --k) {
            const int32_t n = ids[k];
            const double Y3[3] = {conic[n], conic[N + n], conic[2 * N + n]};
            const double dx = mean2d[n] - px, dy = mean2d[N + n] - py;
            const double e = exp(-sigma_of(Y3, dx, dy));
            const double a_raw = opac[n] * e;
            const double alpha = a_raw < prm->alpha_max ? a_raw : prm->alpha_max;
            if (alpha < prm->alpha_min) continue;
            T = T / (1.0 - alpha);                        /* eq. (17) */
            const double c[3] = {colors[n], colors[N + n], colors[2 * N + n]};
            double *o = g9 + 9 * (k - start);
            o[5] += alpha * T * g[0];                     /* eq. (16) */
            o[6] += alpha * T * g[1];
            o[7] += alpha * T * g[2];
            const double gc = g[0] * c[0] + g[1] * c[1] + g[2] * c[2];
            const double dalpha = gc * T - gS / (1.0 - alpha);   /* eq. (18), summed over channels */
            gS += gc * alpha * T;                                 /* S_{n-1} = c_n alpha_n T_n + S_n */
            if (a_raw > prm->alpha_max) continue;                 /* clamped: no gradient to o, sigma */
            o[8] += dalpha * e;                                   /* eq. (19) */
            const double dsigma = dalpha * (-opac[n] * e);        /* eq. (19) */
            const double ddx = delta_flip ? -dx : dx, ddy = delta_flip ? -dy : dy;
            o[0] += dsigma * (Y3[0] * ddx + Y3[1] * ddy);         /* dsigma/dmu' = Y Delta */
            o[1] += dsigma * (Y3[1] * ddx + Y3[2] * ddy);
            o[2] += dsigma * 0.5 * dx * dx;                       /* dsigma/dY = 1/2 Delta Delta^T */
            o[3] += dsigma * 0.5 * dx * dy;
            o[4] += dsigma * 0.5 * dy * dy;
        }
        return;
    }
    /* form 1 */
    int64_t m = 0;
    double *al = (double *)malloc((size_t)(nlast > 0 ? nlast : 1) * 6 * sizeof(double));
    int64_t *pos = (int64_t *)malloc((size_t)(nlast > 0 ? nlast : 1) * sizeof(int64_t));
    double T = 1.0;
    for (int64_t k = start; k < start + nlast; ++k) {
        const int32_t n = ids[k];
        const double Y3[3] = {conic[n], conic[N + n], conic[2 * N + n]};
        const double dx = mean2d[n] - px, dy = mean2d[N + n] - py;
        const double e = exp(-sigma_of(Y3, dx, dy));
        const double a_raw = opac[n] * e;
        const double alpha = a_raw < prm->alpha_max ? a_raw : prm->alpha_max;
        if (alpha < prm->alpha_min) continue;
        al[6 * m + 0] = alpha;
        al[6 * m + 1] = T;                 /* T_n = prod_{m<n} (1 - alpha_m) */
        al[6 * m + 2] = e;
        al[6 * m + 3] = a_raw;
        al[6 * m + 4] = dx;
        al[6 * m + 5] = dy;
        pos[m] = k;
        T *= 1.0 - alpha;
        ++m;
    }
    for (int64_t a = 0; a < m; ++a) {
        const int64_t k = pos[a];
        const int32_t n = ids[k];
        const double alpha = al[6 * a], Tn = al[6 * a + 1], e = al[6 * a + 2], a_raw = al[6 * a + 3];
        const double dx = al[6 * a + 4], dy = al[6 * a + 5];
        const double Y3[3] = {conic[n], conic[N + n], conic[2 * N + n]};
        double *o = g9 + 9 * (k - start);
        double dalpha = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            double S = bg[ch] * T;   /* T = prod over all composited entries: T_final */
            for (int64_t b = a + 1; b < m; ++b)
                S += colors[ch * N + ids[pos[b]]] * al[6 * b] * al[6 * b + 1];
            o[5 + ch] += alpha * Tn * g[ch];
            dalpha += g[ch] * (colors[ch * N + n] * Tn - S / (1.0 - alpha));
        }
        if (a_raw > prm->alpha_max) continue;
        o[8] += dalpha * e;
        const double dsigma = dalpha * (-opac[n] * e);
        const double ddx = delta_flip ? -dx : dx, ddy = delta_flip ? -dy : dy;
        o[0] += dsigma * (Y3[0] * ddx + Y3[1] * ddy);
        o[1] += dsigma * (Y3[1] * ddx + Y3[2] * ddy);
        o[2] += dsigma * 0.5 * dx * dx;
        o[3] += dsigma * 0.5 * dx * dy;
        o[4] += dsigma * 0.5 * dy * dy;
    }
    free(al);
    free(pos);
}

/*
 * Sec. 3.1 over the whole image. dL_dC [3][W*H]; T_final, last from the forward.
 * Per-entry partial gradients are formed tile by tile (each list entry belongs to
 * one tile) and then added into the per-Gaussian outputs in list order, so the
 * result does not depend on the thread count. Outputs are accumulated (+=):
 * dmean2d [2][N], dconic [3][N] = (dY00, dY01, dY11), dcolors [3][N], dopac [N].
 */
void orc_rasterize_bwd(int64_t N, const double *mean2d, const double *conic, const double *colors,
                       const double *opac, int64_t K, const int32_t *ids, const int64_t *ranges,
                       int64_t W, int64_t H, const orc_params *prm, const double *dL_dC,
                       const double *T_final, const int32_t *last, int form,
                       double *dmean2d, double *dconic, double *dcolors, double *dopac)
{
    const int64_t TX = (W + ORC_TILE - 1) / ORC_TILE, TY = (H + ORC_TILE - 1) / ORC_TILE;
    const int64_t HW = W * H;
    double *g9 = (double *)calloc((size_t)(K > 0 ? K : 1) * 9, sizeof(double));
    set_threads(prm);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t tile = 0; tile < TX * TY; ++tile) {
        const int64_t start = ranges[2 * tile];
        const int64_t ty = tile / TX, tx = tile % TX;
        for (int64_t i = ty * ORC_TILE; i < (ty + 1) * ORC_TILE && i < H; ++i)
            for (int64_t j = tx * ORC_TILE; j < (tx + 1) * ORC_TILE && j < W; ++j) {
                const int64_t pix = i * W + j;
                const double g[3] = {dL_dC[pix], dL_dC[HW + pix], dL_dC[2 * HW + pix]};
                pixel_backward(N, mean2d, conic, colors, opac, ids, start, last[pix],
                               (double)j + 0.5, (double)i + 0.5, g, T_final[pix], prm, form,
                               g9 + 9 * start);
            }
    }
    for (int64_t k = 0; k < K; ++k) {
        const int32_t n = ids[k];
        const double *o = g9 + 9 * k;
        dmean2d[n] += o[0];
        dmean2d[N + n] += o[1];
        dconic[n] += o[2];
        dconic[N + n] += o[3];
        dconic[2 * N + n] += o[4];
        dcolors[n] += o[5];
        dcolors[N + n] += o[6];
        dcolors[2 * N + n] += o[7];
        dopac[n] += o[8];
    }
    free(g9);
}

/* ------------------------------------------------------------------ projection gradients */

/* dR/dq for q = (w, x, y, z) (Sec. 3.2.1), each 3x3 row-major. */
static void rot_jacobians(const double *q, double dR[4][9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double Rw[9] = {0, -z, y, z, 0, -x, -y, x, 0};
    const double Rx[9] = {0, y, z, y, -2 * x, -w, z, w, -2 * x};
    const double Ry[9] = {-2 * y, x, w, x, 0, z, -w, z, -2 * y};
    const double Rz[9] = {-2 * z, -w, x, w, -2 * z, y, x, y, 0};
    for (int a = 0; a < 9; ++a) {
        dR[0][a] = 2.0 * Rw[a];
        dR[1][a] = 2.0 * Rx[a];
        dR[2][a] = 2.0 * Ry[a];
        dR[3][a] = 2.0 * Rz[a];
    }
}

/* dL/dSigma' from dL/dY: -Y^T G Y^T (Sec. 3.1, last display). All 2x2 row-major. */
void orc_conic_grad_to_cov2d(const double *Y, const double *G, double *dcov)
{
    double Yt[4], tmp[4];
    tr(Y, Yt, 2, 2);
    mm(Yt, G, tmp, 2, 2, 2);
    mm(tmp, Yt, dcov, 2, 2, 2);
    for (int a = 0; a < 4; ++a) dcov[a] = -dcov[a];
}

/*
 * Sec. 3.2 for each visible Gaussian: given dL/dmu' [2][N] and dL/dY [3][N]
 * (Y00, Y01, Y11 entries of the full-matrix gradient) produce dL/dmu [3][N],
 * dL/ds [3][N], dL/dq [4][N] (accumulated, +=) and, if dTcw is not NULL, the
 * camera-pose gradient dL/dT_cw [4x4 row-major] (accumulated).
 */
void orc_project_bwd(int64_t N, const double *means, const double *quats, const double *scales,
                     const orc_camera *cam, const orc_params *prm,
                     const double *dmean2d, const double *dconic,
                     double *dmeans, double *dscales, double *dquats, double *dTcw)
{
    double P[16], Pt[16];
    proj_matrix(cam, P);
    tr(P, Pt, 4, 4);
    const double w = (double)cam->W, h = (double)cam->H;
    set_threads(prm);
    /* each Gaussian writes only its own outputs; the camera-pose sum runs serially, in
     * Gaussian order */
#pragma omp parallel for schedule(static) if (dTcw == NULL)
    for (int64_t i = 0; i < N; ++i) {
        orc_proj g;
        load_gaussian(N, i, means, quats, scales, &g);
        if (!project_one(cam, prm, &g))
            continue;
        const double dmu2[2] = {dmean2d[i], dmean2d[N + i]};
        const double Gy[4] = {dconic[i], dconic[N + i], dconic[N + i], dconic[2 * N + i]};
        double G2[4];
        orc_conic_grad_to_cov2d(g.Y, Gy, G2);

        /* eq. (23): dL_mu'/dt = 1/2 P^T D^T dL/dmu' */
        const double tw = g.tp[3];
        const double D[8] = {
            w / tw, 0.0, 0.0, -w * g.tp[0] / (tw * tw),
            0.0, h / tw, 0.0, -((prm->errata & ORC_ERRATA_EQ23_W) ? w : h) * g.tp[1] / (tw * tw)};
        double Dt[8], dtp[4], dt[4];
        tr(D, Dt, 2, 4);
        mm(Dt, dmu2, dtp, 4, 2, 1);
        for (int a = 0; a < 4; ++a) dtp[a] *= 0.5;
        mm(Pt, dtp, dt, 4, 4, 1);

        /* eq. (25): dL/dT = G T Sigma^T + G^T T Sigma; dL/dJ = dL/dT R_cw^T */
        double G2t[4], Sigt[9], A1[6], A2[6], dT[6], Rcwt[9], dJ[6];
        tr(G2, G2t, 2, 2);
        tr(g.Sigma, Sigt, 3, 3);
        double TS[6];
        mm(G2, g.T, TS, 2, 2, 3);
        mm(TS, Sigt, A1, 2, 3, 3);
        mm(G2t, g.T, TS, 2, 2, 3);
        mm(TS, g.Sigma, A2, 2, 3, 3);
        for (int a = 0; a < 6; ++a) dT[a] = A1[a] + A2[a];
        tr(cam->R, Rcwt, 3, 3);
        mm(dT, Rcwt, dJ, 2, 3, 3);

        /* dJ/dt (Sec. 3.2) */
        const double tx = g.t[0], ty = g.t[1], tz = g.t[2], fx = cam->fx, fy = cam->fy;
        const double dJx[6] = {0, 0, -fx / (tz * tz), 0, 0, 0};
        const double dJy[6] = {0, 0, 0, 0, 0, -fy / (tz * tz)};
        const double dJz[6] = {-fx / (tz * tz), 0, 2 * fx * tx / (tz * tz * tz),
                               0, -fy / (tz * tz), 2 * fy * ty / (tz * tz * tz)};
        dt[0] += frob(dJ, dJx, 6);
        dt[1] += frob(dJ, dJy, 6);
        dt[2] += frob(dJ, dJz, 6);
        /* dJ/dt_w = 0 */

        /* eq. (28): dL/dmu = R_cw^T dL/dt_xyz; dL/dT_cw = dL/dt [mu; 1]^T */
        double dmu[3];
        mm(Rcwt, dt, dmu, 3, 3, 1);
        for (int a = 0; a < 3; ++a) dmeans[a * N + i] += dmu[a];
        if (dTcw) {
            const double hq[4] = {g.mu[0], g.mu[1], g.mu[2], 1.0};
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c)
                    dTcw[4 * r + c] += dt[r] * hq[c];
            /* R_cw also enters Sigma' through T = J R_cw, so dL/dR_cw gains J^T dL/dT;
             * eq. (28) lists only the path through t. */
            if (!(prm->errata & ORC_ERRATA_EQ28_ONLY)) {
                double Jt[6], JtdT[9];
                tr(g.J, Jt, 2, 3);
                mm(Jt, dT, JtdT, 3, 2, 3);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c)
                        dTcw[4 * r + c] += JtdT[3 * r + c];
            }
        }

        /* eq. (24): dL/dSigma = T^T G T */
        double Tt[6], TtG[6], dSig[9];
        tr(g.T, Tt, 2, 3);
        mm(Tt, G2, TtG, 3, 2, 2);
        mm(TtG, g.T, dSig, 3, 2, 3);

        /* eq. (29): dL/dM = dL/dSigma M + dL/dSigma^T M */
        double dSigt[9], B1[9], B2[9], dM[9];
        tr(dSig, dSigt, 3, 3);
        mm(dSig, g.M, B1, 3, 3, 3);
        mm(dSigt, g.M, B2, 3, 3, 3);
        for (int a = 0; a < 9; ++a) dM[a] = B1[a] + B2[a];

        /* eq. (30): dL/dR = dL/dM S^T, dL/dS = R^T dL/dM */
        const double S[9] = {g.s[0], 0, 0, 0, g.s[1], 0, 0, 0, g.s[2]};
        double St[9], dR[9], Rt[9], dS[9];
        tr(S, St, 3, 3);
        mm(dM, St, dR, 3, 3, 3);
        tr(g.R, Rt, 3, 3);
        mm(Rt, dM, dS, 3, 3, 3);

        /* dR/dq (Sec. 3.2.1) and eq. (31) */
        double dRq[4][9], dq[4];
        rot_jacobians(g.q, dRq);
        for (int a = 0; a < 4; ++a) dq[a] = frob(dR, dRq[a], 9);
        if (prm->normalize_quats) {
            /* through q^ = q / |q|: d q^ / d q = (I - q^ q^T) / |q| */
            const double dot = g.q[0] * dq[0] + g.q[1] * dq[1] + g.q[2] * dq[2] + g.q[3] * dq[3];
            for (int a = 0; a < 4; ++a) dq[a] = (dq[a] - g.q[a] * dot) / g.qn;
        }
        for (int a = 0; a < 4; ++a) dquats[a * N + i] += dq[a];
        for (int a = 0; a < 3; ++a) dscales[a * N + i] += dS[4 * a];
    }
}

/* Exposes the intermediate quantities of one projection for the invariant tests. */
int orc_project_state(const double *mu, const double *q, const double *s, const orc_camera *cam,
                      const orc_params *prm, double *out /* 64 doubles */)
{
    orc_proj g;
    memset(&g, 0, sizeof g);
    memcpy(g.mu, mu, 3 * sizeof(double));
    memcpy(g.q, q, 4 * sizeof(double));
    memcpy(g.s, s, 3 * sizeof(double));
    int ok = project_one(cam, prm, &g);
    memset(out, 0, 64 * sizeof(double));
    memcpy(out + 0, g.R, 9 * sizeof(double));
    memcpy(out + 9, g.Sigma, 9 * sizeof(double));
    memcpy(out + 18, g.t, 4 * sizeof(double));
    memcpy(out + 22, g.tp, 4 * sizeof(double));
    memcpy(out + 26, g.J, 6 * sizeof(double));
    memcpy(out + 32, g.cov2d, 4 * sizeof(double));
    memcpy(out + 36, g.Y, 4 * sizeof(double));
    memcpy(out + 40, g.mean2d, 2 * sizeof(double));
    out[42] = g.depth;
    for (int a = 0; a < 4; ++a) out[43 + a] = (double)g.rect[a];
    out[47] = (double)g.tiles;
    out[48] = g.det;
    return ok;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
