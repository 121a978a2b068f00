/*
 * pmf_oracle.c -- plain FP64 CPU oracle of the PMF-STGR forward model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests and the benchmark's CPU baseline can
 * check the HIP library against a slow, direct transcription of the
 * definitions.  It shares no code, header or constant with the HIP sources.
 *
 * What it computes (arXiv 2503.22139):
 *   - Gaussian kernel, Eq. 4; voxelization sum, Eq. 5 (point samples at voxel
 *     centres, truncated to the ellipsoid m <= k^2);
 *   - low-rank DVF, Eq. 3, with one basis volume per (level, basis, component)
 *     sampled trilinearly at the output voxel centres;
 *   - motion-compensated warp, Eq. 2, I(x) = I_ref(x + d(x));
 *   - X-ray line integral, Eq. 6, discretised as a per-ray midpoint rule over
 *     the ray's chord through the volume box;
 *   - hand-written adjoints of each step (gradients of a scalar loss).
 * Readings of points where the paper is silent (interpolation boundary,
 * geometry, step rule, parameterisation of the covariance) are the ones listed
 * in the design notes of this repository; each function below states the one
 * it uses.
 *
 * Conventions: grid (n, h, centre); voxel (i,j,k) centre = centre +
 * ((i,j,k) - (n-1)/2) h; memory index (i*n1 + j)*n2 + k (axis 2 fastest).
 * Inputs are float32 values promoted to double by the caller.
 *
 * Parallelism: OpenMP loops whose iterations write disjoint outputs; scatters
 * go to per-thread private buffers that are summed afterwards.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int n[3];
    double h[3];
    double c0[3]; /* centre of voxel (0,0,0) */
} ogrid;

static ogrid make_grid(const int *n, const double *h, const double *ctr) {
    ogrid g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.h[a] = h[a];
        g.c0[a] = ctr[a] - 0.5 * (double)(n[a] - 1) * h[a];
    }
    return g;
}

static long gsize(const ogrid *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static void voxel_centre(const ogrid *g, long i, long j, long k, double x[3]) {
    x[0] = g->c0[0] + (double)i * g->h[0];
    x[1] = g->c0[1] + (double)j * g->h[1];
    x[2] = g->c0[2] + (double)k * g->h[2];
}

static int nthreads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int thread_id(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_get_threads(void) { return nthreads(); }

/* ------------------------------------------------------------------ sample3d
 * Trilinear interpolation of a voxel volume at a world point y (Eq. 2 warp,
 * DVF upsampling and the ray-march samples all use it).
 * Reading: the volume is the box of its voxels; outside it (any u_a < -1/2 or
 * u_a > n_a - 1/2 in voxel units) the value is 0 (air); inside, the index is
 * clamped to [0, n-1] so the half-voxel rim takes the edge value.
 * Fills the 8 corner indices and weights; returns 0 when y is outside.
 * dw (optional) receives d(weight)/dy_a for each corner, which is zero along
 * an axis where u is on the clamped rim.
 */
static int trilinear_stencil(const ogrid *g, const double y[3], long idx[8], double w[8],
                             double dw[8][3]) {
    double f[3];
    long i0[3];
    int free_axis[3];
    for (int a = 0; a < 3; ++a) {
        double u = (y[a] - g->c0[a]) / g->h[a];
        if (u < -0.5 || u > (double)g->n[a] - 0.5) return 0;
        double uc = u;
        if (uc < 0.0) uc = 0.0;
        if (uc > (double)(g->n[a] - 1)) uc = (double)(g->n[a] - 1);
        long i = (long)floor(uc);
        if (i > g->n[a] - 2) i = g->n[a] - 2;
        i0[a] = i;
        f[a] = uc - (double)i;
        free_axis[a] = (u > 0.0 && u < (double)(g->n[a] - 1));
    }
    int c = 0;
    for (int dx = 0; dx < 2; ++dx)
        for (int dy = 0; dy < 2; ++dy)
            for (int dz = 0; dz < 2; ++dz, ++c) {
                double wx = dx ? f[0] : 1.0 - f[0];
                double wy = dy ? f[1] : 1.0 - f[1];
                double wz = dz ? f[2] : 1.0 - f[2];
                idx[c] = ((i0[0] + dx) * g->n[1] + (i0[1] + dy)) * (long)g->n[2] + (i0[2] + dz);
                w[c] = wx * wy * wz;
                if (dw) {
                    double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
                    dw[c][0] = free_axis[0] ? sx * wy * wz / g->h[0] : 0.0;
                    dw[c][1] = free_axis[1] ? sy * wx * wz / g->h[1] : 0.0;
                    dw[c][2] = free_axis[2] ? sz * wx * wy / g->h[2] : 0.0;
                }
            }
    return 1;
}

static double sample3d(const double *vol, const ogrid *g, const double y[3]) {
    long idx[8];
    double w[8];
    if (!trilinear_stencil(g, y, idx, w, NULL)) return 0.0;
    double s = 0.0;
    for (int c = 0; c < 8; ++c) s += w[c] * vol[idx[c]];
    return s;
}

/* Exported for tests: S(vol, y) at npts world points, optional gradient. */
void oracle_sample_points(const double *vol, const int *n, const double *h, const double *ctr,
                          const double *pts, long npts, double *out, double *grad) {
    ogrid g = make_grid(n, h, ctr);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < npts; ++p) {
        long idx[8];
        double w[8], dw[8][3];
        double v = 0.0, gr[3] = {0.0, 0.0, 0.0};
        if (trilinear_stencil(&g, pts + 3 * p, idx, w, dw)) {
            for (int c = 0; c < 8; ++c) {
                v += w[c] * vol[idx[c]];
                for (int a = 0; a < 3; ++a) gr[a] += dw[c][a] * vol[idx[c]];
            }
        }
        out[p] = v;
        if (grad)
            for (int a = 0; a < 3; ++a) grad[3 * p + a] = gr[a];
    }
}

/* ------------------------------------------------------------------ Gaussians
 * Eq. 4 with Sigma parameterised by scale s (standard deviations, mm) and a
 * quaternion q = (w, x, y, z) (normalised here): Sigma = R S^2 R^T, so
 * Sigma^{-1} = R diag(s^-2) R^T.  Truncation: only voxels with
 * m = d^T Sigma^{-1} d <= k^2 contribute (k = +inf: untruncated).
 */
typedef struct {
    double mu[3];
    double s[3];
    double qh[4]; /* normalised quaternion */
    double qn;    /* |q| */
    double R[3][3];
    double A[3][3];   /* Sigma^{-1} */
    double ext[3];    /* k * sqrt(Sigma_aa): half-extent of the ellipsoid's bounding box */
} ogauss;

static void gauss_setup(const double *mean, const double *scale, const double *quat, double k,
                        ogauss *G) {
    for (int a = 0; a < 3; ++a) {
        G->mu[a] = mean[a];
        G->s[a] = scale[a];
    }
    double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    G->qn = qn;
    for (int c = 0; c < 4; ++c) G->qh[c] = quat[c] / qn;
    double w = G->qh[0], x = G->qh[1], y = G->qh[2], z = G->qh[3];
    G->R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    G->R[0][1] = 2.0 * (x * y - w * z);
    G->R[0][2] = 2.0 * (x * z + w * y);
    G->R[1][0] = 2.0 * (x * y + w * z);
    G->R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    G->R[1][2] = 2.0 * (y * z - w * x);
    G->R[2][0] = 2.0 * (x * z - w * y);
    G->R[2][1] = 2.0 * (y * z + w * x);
    G->R[2][2] = 1.0 - 2.0 * (x * x + y * y);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int c = 0; c < 3; ++c) acc += G->R[a][c] * G->R[b][c] / (G->s[c] * G->s[c]);
            G->A[a][b] = acc;
        }
    for (int a = 0; a < 3; ++a) {
        double var = 0.0;
        for (int c = 0; c < 3; ++c) var += G->R[a][c] * G->R[a][c] * G->s[c] * G->s[c];
        G->ext[a] = isinf(k) ? INFINITY : k * sqrt(var);
    }
}

/* Voxel index range [lo, hi] on axis a that can hold points of the ellipsoid
 * (its bounding box, widened by one voxel for rounding); the mask test itself
 * decides membership. */
static void gauss_range(const ogauss *G, const ogrid *g, int a, long *lo, long *hi) {
    if (isinf(G->ext[a])) {
        *lo = 0;
        *hi = g->n[a] - 1;
        return;
    }
    double l = floor((G->mu[a] - G->ext[a] - g->c0[a]) / g->h[a]) - 1.0;
    double u = ceil((G->mu[a] + G->ext[a] - g->c0[a]) / g->h[a]) + 1.0;
    if (l < 0.0) l = 0.0;
    if (u > (double)(g->n[a] - 1)) u = (double)(g->n[a] - 1);
    *lo = (long)l;
    *hi = (long)u;
}

static double quad_form(const double A[3][3], const double d[3]) {
    double m = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m += d[a] * A[a][b] * d[b];
    return m;
}

/* Eq. 5: vol[c][j] = sum_i value[i][c] exp(-m_ij / 2) over i with m_ij <= k^2.
 * Reading: point samples at voxel centres; signed values are allowed (the
 * negative-permitting voxelizer of Sec. 2.3.1). */
int oracle_voxelize(const double *mean, const double *scale, const double *quat,
                    const double *value, long m, int nc, const int *n, const double *h,
                    const double *ctr, double k, double *vol) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
    ogauss *G = (ogauss *)malloc(sizeof(ogauss) * (size_t)(m > 0 ? m : 1));
    if (!G) return -1;
    for (long i = 0; i < m; ++i) gauss_setup(mean + 3 * i, scale + 3 * i, quat + 4 * i, k, &G[i]);
    memset(vol, 0, sizeof(double) * (size_t)N * (size_t)nc);
    double k2 = isinf(k) ? INFINITY : k * k;
    /* each thread owns whole x-slices, so writes never collide */
#pragma omp parallel for schedule(dynamic, 1)
    for (long ix = 0; ix < g.n[0]; ++ix) {
        for (long gi = 0; gi < m; ++gi) {
            const ogauss *P = &G[gi];
            long lo[3], hi[3];
            for (int a = 0; a < 3; ++a) gauss_range(P, &g, a, &lo[a], &hi[a]);
            if (ix < lo[0] || ix > hi[0]) continue;
            for (long iy = lo[1]; iy <= hi[1]; ++iy)
                for (long iz = lo[2]; iz <= hi[2]; ++iz) {
                    double x[3], d[3];
                    voxel_centre(&g, ix, iy, iz, x);
                    for (int a = 0; a < 3; ++a) d[a] = x[a] - P->mu[a];
                    double mm = quad_form(P->A, d);
                    if (!(mm <= k2)) continue;
                    double e = exp(-0.5 * mm);
                    long j = (ix * g.n[1] + iy) * (long)g.n[2] + iz;
                    for (int c = 0; c < nc; ++c) vol[(long)c * N + j] += value[gi * nc + c] * e;
                }
        }
    }
    free(G);
    return 0;
}

/* Eq. 5 split by the margin of each pair's mask test, for checks of the
 * binning where several results are correct: a pair whose m lies within
 * `band` of k^2 may fall either side of the mask under float rounding.
 *   inner[c][j] = sum over m <= k^2 - band of value e
 *   edge[c][j]  = sum over k^2 - band < m <= k^2 of value e
 *                 (inner + edge is Eq. 5 itself)
 *   amb[c][j]   = sum over |m - k^2| <= band of |value| e
 *   absum[c][j] = sum over m <= k^2 + band of |value| e
 * Same loop and voxel order as oracle_voxelize. */
int oracle_voxelize_band(const double *mean, const double *scale, const double *quat,
                         const double *value, long m, int nc, const int *n, const double *h,
                         const double *ctr, double k, double band, double *inner, double *edge,
                         double *amb, double *absum) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
    ogauss *G = (ogauss *)malloc(sizeof(ogauss) * (size_t)(m > 0 ? m : 1));
    if (!G) return -1;
    /* the search box must hold the widened ellipsoid m <= k^2 + band */
    const double kw = isinf(k) ? k : sqrt(k * k + band);
    for (long i = 0; i < m; ++i) gauss_setup(mean + 3 * i, scale + 3 * i, quat + 4 * i, kw, &G[i]);
    const size_t bytes = sizeof(double) * (size_t)N * (size_t)nc;
    memset(inner, 0, bytes);
    memset(edge, 0, bytes);
    memset(amb, 0, bytes);
    memset(absum, 0, bytes);
    const double k2 = isinf(k) ? INFINITY : k * k;
#pragma omp parallel for schedule(dynamic, 1)
    for (long ix = 0; ix < g.n[0]; ++ix) {
        for (long gi = 0; gi < m; ++gi) {
            const ogauss *P = &G[gi];
            long lo[3], hi[3];
            for (int a = 0; a < 3; ++a) gauss_range(P, &g, a, &lo[a], &hi[a]);
            if (ix < lo[0] || ix > hi[0]) continue;
            for (long iy = lo[1]; iy <= hi[1]; ++iy)
                for (long iz = lo[2]; iz <= hi[2]; ++iz) {
                    double x[3], d[3];
                    voxel_centre(&g, ix, iy, iz, x);
                    for (int a = 0; a < 3; ++a) d[a] = x[a] - P->mu[a];
                    const double mm = quad_form(P->A, d);
                    if (!(mm <= k2 + band)) continue;
                    const double e = exp(-0.5 * mm);
                    const long j = (ix * g.n[1] + iy) * (long)g.n[2] + iz;
                    for (int c = 0; c < nc; ++c) {
                        const double v = value[gi * nc + c];
                        const long q = (long)c * N + j;
                        absum[q] += fabs(v) * e;
                        if (mm <= k2 - band) inner[q] += v * e;
                        else if (mm <= k2) edge[q] += v * e;
                        if (fabs(mm - k2) <= band) amb[q] += fabs(v) * e;
                    }
                }
        }
    }
    free(G);
    return 0;
}

/* Gradient of a scalar loss L through Eq. 5, given g_vol = dL/dvol [c][N].
 * With the truncation mask held fixed, for Gaussian i and each in-mask voxel j
 * (e = exp(-m/2), G_j = sum_c value[i][c] g_vol[c][j], d_j = x_j - mu):
 *   dL/dvalue[i][c] = sum_j g_vol[c][j] e
 *   dL/dmu          = sum_j G_j e A d_j
 *   dL/dA = M       = -1/2 sum_j G_j e d_j d_j^T
 *   A = R diag(s^-2) R^T  =>  dL/ds_k = -2 s_k^-3 (R^T M R)_kk,
 *                             dL/dR   = 2 M R diag(s^-2)
 *   R(q^) as in gauss_setup  =>  dL/dq^ by differentiating its nine entries,
 *   q^ = q/|q|               =>  dL/dq = (g - q^ (q^.g)) / |q|.            */
int oracle_voxelize_bwd(const double *mean, const double *scale, const double *quat,
                        const double *value, long m, int nc, const int *n, const double *h,
                        const double *ctr, double k, const double *g_vol, double *g_mean,
                        double *g_scale, double *g_quat, double *g_value) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
    double k2 = isinf(k) ? INFINITY : k * k;
#pragma omp parallel for schedule(dynamic, 16)
    for (long gi = 0; gi < m; ++gi) {
        ogauss P;
        gauss_setup(mean + 3 * gi, scale + 3 * gi, quat + 4 * gi, k, &P);
        long lo[3], hi[3];
        for (int a = 0; a < 3; ++a) gauss_range(&P, &g, a, &lo[a], &hi[a]);
        double gv[64];
        double gmu[3] = {0, 0, 0};
        double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        double *gvp = nc <= 64 ? gv : (double *)calloc((size_t)nc, sizeof(double));
        for (int c = 0; c < nc; ++c) gvp[c] = 0.0;
        for (long ix = lo[0]; ix <= hi[0]; ++ix)
            for (long iy = lo[1]; iy <= hi[1]; ++iy)
                for (long iz = lo[2]; iz <= hi[2]; ++iz) {
                    double x[3], d[3];
                    voxel_centre(&g, ix, iy, iz, x);
                    for (int a = 0; a < 3; ++a) d[a] = x[a] - P.mu[a];
                    double mm = quad_form(P.A, d);
                    if (!(mm <= k2)) continue;
                    double e = exp(-0.5 * mm);
                    long j = (ix * g.n[1] + iy) * (long)g.n[2] + iz;
                    double Gj = 0.0;
                    for (int c = 0; c < nc; ++c) {
                        double gc = g_vol[(long)c * N + j];
                        gvp[c] += gc * e;
                        Gj += value[gi * nc + c] * gc;
                    }
                    double t = Gj * e;
                    for (int a = 0; a < 3; ++a) {
                        double Ad = P.A[a][0] * d[0] + P.A[a][1] * d[1] + P.A[a][2] * d[2];
                        gmu[a] += t * Ad;
                        for (int b = 0; b < 3; ++b) M[a][b] += -0.5 * t * d[a] * d[b];
                    }
                }
        for (int c = 0; c < nc; ++c) g_value[gi * nc + c] = gvp[c];
        if (gvp != gv) free(gvp);
        for (int a = 0; a < 3; ++a) g_mean[3 * gi + a] = gmu[a];
        /* R^T M R diagonal -> scale gradient */
        double MR[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                MR[a][b] = M[a][0] * P.R[0][b] + M[a][1] * P.R[1][b] + M[a][2] * P.R[2][b];
        for (int kk = 0; kk < 3; ++kk) {
            double d = P.R[0][kk] * MR[0][kk] + P.R[1][kk] * MR[1][kk] + P.R[2][kk] * MR[2][kk];
            g_scale[3 * gi + kk] = -2.0 * d / (P.s[kk] * P.s[kk] * P.s[kk]);
        }
        double GR[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) GR[a][b] = 2.0 * MR[a][b] / (P.s[b] * P.s[b]);
        double w = P.qh[0], x = P.qh[1], y = P.qh[2], z = P.qh[3];
        /* derivative of each rotation-matrix entry with respect to (w,x,y,z) */
        double gq[4];
        gq[0] = 2.0 * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] +
                       x * GR[2][1]);
        gq[1] = 2.0 * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2.0 * x * GR[1][1] -
                       w * GR[1][2] + z * GR[2][0] + w * GR[2][1] - 2.0 * x * GR[2][2]);
        gq[2] = 2.0 * (-2.0 * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] +
                       z * GR[1][2] - w * GR[2][0] + z * GR[2][1] - 2.0 * y * GR[2][2]);
        gq[3] = 2.0 * (-2.0 * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] -
                       2.0 * z * GR[1][1] + y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
        double dot = gq[0] * P.qh[0] + gq[1] * P.qh[1] + gq[2] * P.qh[2] + gq[3] * P.qh[3];
        for (int c = 0; c < 4; ++c) g_quat[4 * gi + c] = (gq[c] - P.qh[c] * dot) / P.qn;
    }
    return 0;
}

/* Brute-force Eq. 5 at arbitrary voxel indices (every Gaussian tested), used
 * for sampled checks of large grids.  idx: flat voxel indices. */
int oracle_voxelize_points(const double *mean, const double *scale, const double *quat,
                           const double *value, long m, int nc, const int *n, const double *h,
                           const double *ctr, double k, const long *idx, long npts, double *out) {
    ogrid g = make_grid(n, h, ctr);
    ogauss *G = (ogauss *)malloc(sizeof(ogauss) * (size_t)(m > 0 ? m : 1));
    if (!G) return -1;
    for (long i = 0; i < m; ++i) gauss_setup(mean + 3 * i, scale + 3 * i, quat + 4 * i, k, &G[i]);
    double k2 = isinf(k) ? INFINITY : k * k;
#pragma omp parallel for schedule(dynamic, 4)
    for (long p = 0; p < npts; ++p) {
        long j = idx[p];
        long iz = j % g.n[2], iy = (j / g.n[2]) % g.n[1], ix = j / ((long)g.n[1] * g.n[2]);
        double x[3];
        voxel_centre(&g, ix, iy, iz, x);
        for (int c = 0; c < nc; ++c) out[p * nc + c] = 0.0;
        for (long gi = 0; gi < m; ++gi) {
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = x[a] - G[gi].mu[a];
            double mm = quad_form(G[gi].A, d);
            if (!(mm <= k2)) continue;
            double e = exp(-0.5 * mm);
            for (int c = 0; c < nc; ++c) out[p * nc + c] += value[gi * nc + c] * e;
        }
    }
    free(G);
    return 0;
}

/* -------------------------------------------------------------------- Eq. 3
 * d_k(x, p_v) = sum_l sum_b w[v][l][b][k] S(E_l[b*3+k], x), with every level's
 * basis volume E_l ([3B][n_l], channel b*3+k) sampled trilinearly (sample3d)
 * at the output voxel centres x.  dvf: [V][3][N].
 * Reading: "three MBCs per Cartesian direction" become B bases per level and
 * component; each level has its own grid over the same field of view. */
typedef struct {
    ogrid g;
    const double *E;
} olevel;

int oracle_combine(int L, int B, const double *const *bases, const int *lvl_n,
                   const double *lvl_h, const double *lvl_ctr, const double *coeff, int V,
                   const int *n, const double *h, const double *ctr, double *dvf) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
    olevel *lv = (olevel *)malloc(sizeof(olevel) * (size_t)L);
    for (int l = 0; l < L; ++l) {
        lv[l].g = make_grid(lvl_n + 3 * l, lvl_h + 3 * l, lvl_ctr + 3 * l);
        lv[l].E = bases[l];
    }
#pragma omp parallel for schedule(static)
    for (long j = 0; j < N; ++j) {
        long iz = j % g.n[2], iy = (j / g.n[2]) % g.n[1], ix = j / ((long)g.n[1] * g.n[2]);
        double x[3];
        voxel_centre(&g, ix, iy, iz, x);
        for (int v = 0; v < V; ++v)
            for (int kk = 0; kk < 3; ++kk) dvf[((long)v * 3 + kk) * N + j] = 0.0;
        for (int l = 0; l < L; ++l) {
            long Nl = gsize(&lv[l].g);
            for (int b = 0; b < B; ++b)
                for (int kk = 0; kk < 3; ++kk) {
                    double s = sample3d(lv[l].E + (long)(b * 3 + kk) * Nl, &lv[l].g, x);
                    for (int v = 0; v < V; ++v)
                        dvf[((long)v * 3 + kk) * N + j] +=
                            coeff[(((long)v * L + l) * B + b) * 3 + kk] * s;
                }
        }
    }
    free(lv);
    return 0;
}

/* Adjoint of oracle_combine given g_dvf [V][3][N]:
 *   g_coeff[v][l][b][k] = sum_j g_dvf[v][k][j] S(E_l[b*3+k], x_j)
 *   g_E_l[b*3+k]       = sum_v w[v][l][b][k] S_l^T(g_dvf[v][k])
 * where S_l^T spreads each value back onto the 8 corners with the trilinear
 * weights.  One (level, channel) per loop iteration, so writes never collide. */
int oracle_combine_bwd(int L, int B, const double *const *bases, const int *lvl_n,
                       const double *lvl_h, const double *lvl_ctr, const double *coeff, int V,
                       const int *n, const double *h, const double *ctr, const double *g_dvf,
                       double *const *g_bases, double *g_coeff) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
    int C = 3 * B;
#pragma omp parallel for schedule(dynamic, 1)
    for (int lc = 0; lc < L * C; ++lc) {
        int l = lc / C, c = lc % C, b = c / 3, kk = c % 3;
        ogrid gl = make_grid(lvl_n + 3 * l, lvl_h + 3 * l, lvl_ctr + 3 * l);
        long Nl = gsize(&gl);
        const double *E = bases[l] + (long)c * Nl;
        double *gE = g_bases[l] + (long)c * Nl;
        memset(gE, 0, sizeof(double) * (size_t)Nl);
        for (int v = 0; v < V; ++v) {
            double w = coeff[(((long)v * L + l) * B + b) * 3 + kk];
            const double *gd = g_dvf + ((long)v * 3 + kk) * N;
            double gw = 0.0;
            for (long j = 0; j < N; ++j) {
                long iz = j % g.n[2], iy = (j / g.n[2]) % g.n[1], ix = j / ((long)g.n[1] * g.n[2]);
                double x[3];
                voxel_centre(&g, ix, iy, iz, x);
                long idx[8];
                double wt[8];
                if (!trilinear_stencil(&gl, x, idx, wt, NULL)) continue;
                double s = 0.0;
                for (int q = 0; q < 8; ++q) {
                    s += wt[q] * E[idx[q]];
                    gE[idx[q]] += w * wt[q] * gd[j];
                }
                gw += gd[j] * s;
            }
            g_coeff[(((long)v * L + l) * B + b) * 3 + kk] = gw;
        }
    }
    return 0;
}

/* -------------------------------------------------------------------- Eq. 2
 * out[v][j] = S(ref, x_j + dvf[v][:, j]) (pull-back warp, trilinear). */
int oracle_warp(const double *ref, const int *n, const double *h, const double *ctr,
                const double *dvf, int V, double *out) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
#pragma omp parallel for schedule(static)
    for (long j = 0; j < N; ++j) {
        long iz = j % g.n[2], iy = (j / g.n[2]) % g.n[1], ix = j / ((long)g.n[1] * g.n[2]);
        double x[3];
        voxel_centre(&g, ix, iy, iz, x);
        for (int v = 0; v < V; ++v) {
            double y[3];
            for (int a = 0; a < 3; ++a) y[a] = x[a] + dvf[((long)v * 3 + a) * N + j];
            out[(long)v * N + j] = sample3d(ref, &g, y);
        }
    }
    return 0;
}

/* Adjoint of oracle_warp given g_out [V][N]:
 *   g_ref     = sum_v sum_j g_out[v][j] * (trilinear weights at y_vj)
 *   g_dvf[v][a][j] = g_out[v][j] * dS/dy_a(ref, y_vj)                     */
int oracle_warp_bwd(const double *ref, const int *n, const double *h, const double *ctr,
                    const double *dvf, int V, const double *g_out, double *g_ref, double *g_dvf) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
    int T = nthreads();
    double *priv = (double *)calloc((size_t)T * (size_t)N, sizeof(double));
    if (!priv) return -1;
#pragma omp parallel
    {
        double *mine = priv + (size_t)thread_id() * (size_t)N;
#pragma omp for schedule(static)
        for (long j = 0; j < N; ++j) {
            long iz = j % g.n[2], iy = (j / g.n[2]) % g.n[1], ix = j / ((long)g.n[1] * g.n[2]);
            double x[3];
            voxel_centre(&g, ix, iy, iz, x);
            for (int v = 0; v < V; ++v) {
                double y[3];
                for (int a = 0; a < 3; ++a) y[a] = x[a] + dvf[((long)v * 3 + a) * N + j];
                long idx[8];
                double w[8], dw[8][3];
                double go = g_out[(long)v * N + j];
                double gr[3] = {0.0, 0.0, 0.0};
                if (trilinear_stencil(&g, y, idx, w, dw)) {
                    for (int c = 0; c < 8; ++c) {
                        mine[idx[c]] += go * w[c];
                        for (int a = 0; a < 3; ++a) gr[a] += dw[c][a] * ref[idx[c]];
                    }
                }
                for (int a = 0; a < 3; ++a) g_dvf[((long)v * 3 + a) * N + j] = go * gr[a];
            }
        }
    }
    for (long j = 0; j < N; ++j) {
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += priv[(size_t)t * (size_t)N + j];
        g_ref[j] = s;
    }
    free(priv);
    return 0;
}

/* ------------------------------------------------------------ Eq. 6 (rays)
 * Geometry (reading of the full-fan circular scan of Sec. 2.3.3 / Table I):
 * rotation about z, source o = SAD (cos t, sin t, 0), flat detector centred
 * at -(SDD - SAD)(cos t, sin t, 0) with axes e_u = (-sin t, cos t, 0),
 * e_v = (0, 0, 1); one ray from o through each pixel centre
 *   p = c_d + (iu - (nu-1)/2 + off_u) du e_u + (iv - (nv-1)/2 + off_v) dv e_v.
 * Line integral (Eq. 6) over the ray's chord [t_n, t_f] through the volume box
 * (t_n >= 0), midpoint rule with N = max(1, ceil(L / dt)) equal steps,
 * delta = L / N, t_s = t_n + (s + 1/2) delta:  P = delta sum_s S(I, o + t_s d).
 * cone[] = {sad, sdd, du, dv, off_u, off_v, step}; step <= 0 means 0.5 min(h). */
typedef struct {
    double o[3], d[3];
    double tn, tf;
    long nsteps;
    double delta;
} oray;

static void make_ray(const ogrid *g, const double *cone, int nu, int nv, double theta, int iu,
                     int iv, oray *r) {
    double sad = cone[0], sdd = cone[1], du = cone[2], dv = cone[3];
    double ct = cos(theta), st = sin(theta);
    double o[3] = {sad * ct, sad * st, 0.0};
    double cd[3] = {-(sdd - sad) * ct, -(sdd - sad) * st, 0.0};
    double eu[3] = {-st, ct, 0.0};
    double ev[3] = {0.0, 0.0, 1.0};
    double a = ((double)iu - 0.5 * (double)(nu - 1) + cone[4]) * du;
    double b = ((double)iv - 0.5 * (double)(nv - 1) + cone[5]) * dv;
    double p[3], d[3], len = 0.0;
    for (int k = 0; k < 3; ++k) {
        p[k] = cd[k] + a * eu[k] + b * ev[k];
        d[k] = p[k] - o[k];
        len += d[k] * d[k];
    }
    len = sqrt(len);
    for (int k = 0; k < 3; ++k) {
        r->o[k] = o[k];
        r->d[k] = d[k] / len;
    }
    /* slab intersection with the box of the voxels */
    double t0 = -INFINITY, t1 = INFINITY;
    int miss = 0;
    for (int k = 0; k < 3; ++k) {
        double lo = g->c0[k] - 0.5 * g->h[k];
        double hi = g->c0[k] + ((double)g->n[k] - 0.5) * g->h[k];
        if (r->d[k] == 0.0) {
            if (r->o[k] < lo || r->o[k] > hi) miss = 1;
            continue;
        }
        double ta = (lo - r->o[k]) / r->d[k], tb = (hi - r->o[k]) / r->d[k];
        if (ta > tb) {
            double t = ta;
            ta = tb;
            tb = t;
        }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (t0 < 0.0) t0 = 0.0;
    double L = miss ? 0.0 : t1 - t0;
    if (!(L > 0.0)) L = 0.0;
    r->tn = t0;
    r->tf = t0 + L;
    double step = cone[6];
    if (!(step > 0.0)) {
        step = g->h[0];
        if (g->h[1] < step) step = g->h[1];
        if (g->h[2] < step) step = g->h[2];
        step *= 0.5;
    }
    if (L > 0.0) {
        long ns = (long)ceil(L / step);
        if (ns < 1) ns = 1;
        r->nsteps = ns;
        r->delta = L / (double)ns;
    } else {
        r->nsteps = 0;
        r->delta = 0.0;
    }
}

/* Exported for tests: chord [tn, tf], step count and step of each pixel of
 * one view; out has 4 doubles per pixel (tn, tf, nsteps, delta). */
void oracle_ray_info(const int *n, const double *h, const double *ctr, const double *cone, int nu,
                     int nv, double theta, double *out) {
    ogrid g = make_grid(n, h, ctr);
    for (int iv = 0; iv < nv; ++iv)
        for (int iu = 0; iu < nu; ++iu) {
            oray r;
            make_ray(&g, cone, nu, nv, theta, iu, iv, &r);
            double *o = out + 4 * ((long)iv * nu + iu);
            o[0] = r.tn;
            o[1] = r.tf;
            o[2] = (double)r.nsteps;
            o[3] = r.delta;
        }
}

static double march(const double *vol, const ogrid *g, const oray *r) {
    double acc = 0.0;
    for (long s = 0; s < r->nsteps; ++s) {
        double t = r->tn + ((double)s + 0.5) * r->delta;
        double y[3] = {r->o[0] + t * r->d[0], r->o[1] + t * r->d[1], r->o[2] + t * r->d[2]};
        acc += sample3d(vol, g, y);
    }
    return acc * r->delta;
}

/* proj[v][iv][iu]; volume of view v at vol + v*vol_stride (stride 0: shared). */
int oracle_project(const double *vol, long vol_stride, const int *n, const double *h,
                   const double *ctr, const double *cone, int nu, int nv, const double *angles,
                   int V, double *proj) {
    ogrid g = make_grid(n, h, ctr);
    long npix = (long)nu * nv;
#pragma omp parallel for schedule(dynamic, 64)
    for (long q = 0; q < (long)V * npix; ++q) {
        int v = (int)(q / npix);
        long p = q % npix;
        oray r;
        make_ray(&g, cone, nu, nv, angles[v], (int)(p % nu), (int)(p / nu), &r);
        proj[q] = march(vol + (long)v * vol_stride, &g, &r);
    }
    return 0;
}

/* Selected rays only: rays[3*i] = (view, iu, iv). */
int oracle_project_rays(const double *vol, long vol_stride, const int *n, const double *h,
                        const double *ctr, const double *cone, int nu, int nv,
                        const double *angles, const long *rays, long nrays, double *out) {
    ogrid g = make_grid(n, h, ctr);
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < nrays; ++i) {
        oray r;
        long v = rays[3 * i];
        make_ray(&g, cone, nu, nv, angles[v], (int)rays[3 * i + 1], (int)rays[3 * i + 2], &r);
        out[i] = march(vol + v * vol_stride, &g, &r);
    }
    return 0;
}

/* Adjoint of oracle_project: g_vol[v] (or the single g_vol when vol_stride is
 * 0, summed over views) = sum over rays and samples of
 * delta * g_proj(r) * (trilinear weights at the sample). */
int oracle_project_bwd(const double *g_proj, const int *n, const double *h, const double *ctr,
                       const double *cone, int nu, int nv, const double *angles, int V,
                       double *g_vol, long vol_stride) {
    ogrid g = make_grid(n, h, ctr);
    long N = gsize(&g);
    long npix = (long)nu * nv;
    int T = nthreads();
    double *priv = (double *)malloc(sizeof(double) * (size_t)T * (size_t)N);
    if (!priv) return -1;
    long nout = vol_stride ? (long)V : 1;
    for (long i = 0; i < nout; ++i) memset(g_vol + i * (vol_stride ? vol_stride : 0), 0,
                                            sizeof(double) * (size_t)N);
    for (int v = 0; v < V; ++v) {
        memset(priv, 0, sizeof(double) * (size_t)T * (size_t)N);
#pragma omp parallel
        {
            double *mine = priv + (size_t)thread_id() * (size_t)N;
#pragma omp for schedule(dynamic, 64)
            for (long p = 0; p < npix; ++p) {
                oray r;
                make_ray(&g, cone, nu, nv, angles[v], (int)(p % nu), (int)(p / nu), &r);
                double gp = g_proj[(long)v * npix + p] * r.delta;
                for (long s = 0; s < r.nsteps; ++s) {
                    double t = r.tn + ((double)s + 0.5) * r.delta;
                    double y[3] = {r.o[0] + t * r.d[0], r.o[1] + t * r.d[1], r.o[2] + t * r.d[2]};
                    long idx[8];
                    double w[8];
                    if (!trilinear_stencil(&g, y, idx, w, NULL)) continue;
                    for (int c = 0; c < 8; ++c) mine[idx[c]] += gp * w[c];
                }
            }
        }
        double *dst = g_vol + (long)v * vol_stride;
#pragma omp parallel for schedule(static)
        for (long j = 0; j < N; ++j) {
            double s = 0.0;
            for (int t = 0; t < T; ++t) s += priv[(size_t)t * (size_t)N + j];
            dst[j] += s;
        }
    }
    free(priv);
    return 0;
}

/* ------------------------------------------------------------------ loss
 * L2 projection loss over a batch of V views (the batch mean mirrors the
 * 1/N_batch of Eq. 12; the L2 norm is the data term of Eq. 1):
 *   L = (1/V) sum_v sum_r (P - T)^2,  g_P = 2 (P - T) / V.            */
double oracle_l2_loss(const double *proj, const double *target, long npix, int V, double *g) {
    double L = 0.0;
    long tot = npix * (long)V;
    for (long i = 0; i < tot; ++i) {
        double r = proj[i] - target[i];
        L += r * r;
        if (g) g[i] = 2.0 * r / (double)V;
    }
    return L / (double)V;
}
