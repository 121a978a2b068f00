/*
 * pmf.h -- C ABI of libpmf.so, the MI355X (gfx950) implementation of the
 * differentiable forward model of PMF-STGR (arXiv 2503.22139, Sec. 2.3):
 *
 *   reference Gaussians --voxelize (Eq. 4-5)--> I_ref
 *   MBC Gaussians       --voxelize, signed (Sec. 2.3.1)--> basis volumes E_l
 *   E_l, w(p)           --combine (Eq. 3)--> DVF d(x, p)
 *   I_ref, d            --warp (Eq. 2)--> I(x, p)
 *   I(x, p)             --cone-beam line integrals (Eq. 6)--> DRR
 *
 * and the adjoint (gradient) of every step.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every float pointer is a DEVICE pointer to contiguous float32 data owned
 *    by the caller, unless the comment says "host".  The library never
 *    allocates, frees or retains memory: scratch space is a caller-provided
 *    device buffer whose size the matching *_workspace() query returns (the
 *    one exception, pmf_tv_loss_noalloc, uses a small static device array).
 *  - Every call enqueues work on `stream` (a hipStream_t; NULL = the legacy
 *    default stream) and returns without waiting.  Host-side argument checks
 *    run first; on failure nothing is enqueued.
 *  - Forward outputs and gradient outputs are OVERWRITTEN (not accumulated).
 *  - Return value: PMF_OK (0) or a negative pmf_status; pmf_last_error()
 *    gives a message (thread-local, valid until the next call on the thread).
 *  - Volumes: grid (n, h, center); voxel (i,j,k) has its centre at
 *    center + ((i,j,k) - (n-1)/2) * h (mm); memory order [n0][n1][n2], axis 2
 *    (the rotation axis z) fastest.  Multi-channel volumes are [C][n0][n1][n2].
 *    Every n_a >= 2, every h_a > 0, and n0*n1*n2 < 2^31.
 *  - Interpolation (warp, DVF upsampling, ray samples) is trilinear over the
 *    voxel centres; a point beyond the box of the voxels (more than half a
 *    voxel past the outer centres) reads 0, and a point on that half-voxel rim
 *    reads the edge voxel.
 *  - Projections are [V][nv][nu], u fastest.
 *
 * Concurrency: calls are reentrant; two calls that write the same buffer, or
 * share one workspace, must be ordered on one stream.
 */
#ifndef PMF_H
#define PMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMF_VERSION 100 /* 1.0.0 */

typedef enum {
    PMF_OK = 0,
    PMF_EINVAL = -1,       /* invalid argument (null pointer, bad size or geometry) */
    PMF_EHIP = -2,         /* a HIP runtime call or kernel launch failed */
    PMF_EWORKSPACE = -3,   /* workspace missing or smaller than the query returned */
    PMF_EUNSUPPORTED = -4  /* valid but outside what this library supports (e.g. C > 16) */
} pmf_status;

/* Voxel grid.  n: voxels per axis; h: spacing (mm); center: world position of
 * the grid centre (mm). */
typedef struct {
    int32_t n[3];
    float h[3];
    float center[3];
} pmf_grid_t;

/* Circular cone-beam geometry with a flat detector (Sec. 2.3.3, Table I).
 * The gantry rotates about z; at angle t the source sits at
 * SAD (cos t, sin t, 0) and the detector centre at -(SDD - SAD)(cos t, sin t, 0);
 * detector axes e_u = (-sin t, cos t, 0), e_v = (0, 0, 1).  Pixel (iu, iv) is
 * centred at (iu - (nu-1)/2 + off_u) du along e_u and (iv - (nv-1)/2 + off_v) dv
 * along e_v; one ray joins the source to each pixel centre.  The line integral
 * (Eq. 6) over the ray's chord [t_n, t_f] through the volume box is taken with
 * the midpoint rule on N = max(1, ceil((t_f - t_n)/step)) equal sub-intervals.
 * step <= 0 selects half the smallest voxel spacing.  Requires 0 < SAD < SDD
 * and the volume box to lie strictly inside the source circle.  Calls that
 * project (pmf_project*, pmf_warp_project*) also require n1*n2 < 2^24 and
 * n0*n1*n2 < 2^30 (PMF_EUNSUPPORTED otherwise). */
typedef struct {
    float sad, sdd;
    int32_t nu, nv;
    float du, dv;
    float off_u, off_v;
    float step;
} pmf_cone_t;

/* A set of m anisotropic Gaussians, Eq. 4, with Sigma = R(q) diag(scale^2) R(q)^T.
 * mean [m][3] mm; scale [m][3] mm (standard deviations, > 0); quat [m][4]
 * (w, x, y, z), any non-zero norm (normalised inside); value [m][c]: the
 * density rho (c = 1) or signed motion-basis values (c channels, Sec. 2.3.1).
 * m = 0 is allowed. */
typedef struct {
    const float *mean;
    const float *scale;
    const float *quat;
    const float *value;
    int64_t m;
    int32_t c;
} pmf_gauss_t;

/* Gradients with respect to a pmf_gauss_t's arrays (same shapes). */
typedef struct {
    float *mean;
    float *scale;
    float *quat;
    float *value;
} pmf_gauss_grad_t;

/* ------------------------------------------------------------------ info */
int pmf_version(void);
const char *pmf_last_error(void);

/* ------------------------------------------------------------ voxelize
 * Eq. 5 on the voxel centres (point samples):
 *   vol[c][j] = sum_i value[i][c] exp(-m_ij / 2),   m_ij = d^T Sigma_i^-1 d,
 *   d = x_j - mean_i, over the Gaussians with m_ij <= trunc_k^2
 *   (trunc_k = INFINITY: every Gaussian everywhere).
 * Values may be negative (the negative-permitting voxelizer of Sec. 2.3.1).
 * vol: [c][N] output.  Needs the workspace from pmf_voxelize_workspace().
 * Supports c <= 16. */
size_t pmf_voxelize_workspace(int64_t m, int32_t c, const pmf_grid_t *grid);
int pmf_voxelize(const pmf_gauss_t *g, const pmf_grid_t *grid, float trunc_k, float *vol,
                 void *ws, size_t ws_bytes, void *stream);

/* Gradient of a scalar loss through pmf_voxelize given g_vol = dL/dvol [c][N],
 * with the truncation mask held fixed: writes dL/dmean, dL/dscale, dL/dquat
 * (through the normalisation of q) and dL/dvalue.  No workspace. */
int pmf_voxelize_bwd(const pmf_gauss_t *g, const pmf_grid_t *grid, float trunc_k,
                     const float *g_vol, const pmf_gauss_grad_t *grad, void *stream);

/* ------------------------------------------------------- combine DVF (Eq. 3)
 * Low-rank motion model with L levels of B bases per Cartesian component
 * (the paper uses L = 3 levels, one basis per level and component):
 *   dvf[v][k][j] = sum_l sum_b coeff[v][l][b][k] * S(bases[l][b*3 + k], x_j)
 * where S samples level l's volume (grid lvl[l], [3B][N_l]) trilinearly at the
 * output voxel centre x_j (upsampling; identity when lvl[l] equals out).
 * bases: HOST array of L device pointers; lvl: HOST array of L grids;
 * coeff: device [V][L][B][3]; dvf: device [V][3][N] (mm).
 * Supports L <= 4, B <= 4. */
int pmf_combine_dvf(int L, int B, const float *const *bases, const pmf_grid_t *lvl,
                    const float *coeff, int V, const pmf_grid_t *out, float *dvf, void *stream);

/* Adjoint of pmf_combine_dvf given g_dvf [V][3][N]:
 *   g_coeff[v][l][b][k] = sum_j g_dvf[v][k][j] S(bases[l][b*3+k], x_j)
 *   g_bases[l][b*3+k]   = sum_v coeff[v][l][b][k] S_l^T g_dvf[v][k]
 * g_bases: HOST array of L device pointers ([3B][N_l] each).
 * Needs the workspace from pmf_combine_dvf_bwd_workspace(). */
size_t pmf_combine_dvf_bwd_workspace(int L, int B, const pmf_grid_t *lvl, int V,
                                     const pmf_grid_t *out);
int pmf_combine_dvf_bwd(int L, int B, const float *const *bases, const pmf_grid_t *lvl,
                        const float *coeff, int V, const pmf_grid_t *out, const float *g_dvf,
                        float *const *g_bases, float *g_coeff, void *ws, size_t ws_bytes,
                        void *stream);

/* ------------------------------------------------------------ warp (Eq. 2)
 * Pull-back warp of the reference volume by each view's DVF:
 *   out[v][j] = S(ref, x_j + dvf[v][:, j]).
 * ref [N]; dvf [V][3][N] (mm); out [V][N]. */
int pmf_warp(const float *ref, const pmf_grid_t *grid, const float *dvf, int V, float *out,
             void *stream);

/* Adjoint of pmf_warp given g_out [V][N]:
 *   g_ref = sum_v S_v^T g_out[v]   (trilinear weights at x_j + dvf),  [N]
 *   g_dvf[v][a][j] = g_out[v][j] dS/dy_a(ref, x_j + dvf[v][:, j]),    [V][3][N]
 * dS/dy_a is the derivative of the trilinear interpolant inside the
 * voxel-centre hull and 0 on the half-voxel rim and outside; the cell of a
 * point is decided by its displacement, so a point on a cell face takes the
 * side its displacement puts it on (none: the cell that starts at its voxel).
 * g_ref is summed in 64-bit fixed point (each term exact to 2^-40 of the
 * largest |g_out|), so it repeats bit for bit.  Needs the workspace from
 * pmf_warp_bwd_workspace() (8 bytes per voxel). */
size_t pmf_warp_bwd_workspace(const pmf_grid_t *grid);
int pmf_warp_bwd(const float *ref, const pmf_grid_t *grid, const float *dvf, int V,
                 const float *g_out, float *g_ref, float *g_dvf, void *ws, size_t ws_bytes,
                 void *stream);

/* --------------------------------------------------- projection (Eq. 6)
 * DRRs of V views: proj[v][iv][iu] = delta * sum_s S(vol_v, o + t_s d),
 * t_s = t_n + (s + 1/2) delta (geometry in pmf_cone_t).
 * vol_v = vol + v * vol_stride (floats); vol_stride = 0 projects one volume
 * in every view.  angles: device [V] (rad).  proj: [V][nv][nu]. */
int pmf_project(const float *vol, int64_t vol_stride, const pmf_grid_t *grid,
                const pmf_cone_t *cone, const float *angles, int V, float *proj, void *stream);

/* Exact adjoint (back-projection) of pmf_project given g_proj [V][nv][nu]:
 * g_vol_v = P_v^T g_proj[v].  vol_stride = N writes one volume per view
 * ([V][N]); vol_stride = 0 writes their sum ([N]).
 * Needs the workspace from pmf_project_bwd_workspace(). */
size_t pmf_project_bwd_workspace(const pmf_grid_t *grid, const pmf_cone_t *cone, int V);
int pmf_project_bwd(const float *g_proj, const pmf_grid_t *grid, const pmf_cone_t *cone,
                    const float *angles, int V, float *g_vol, int64_t vol_stride, void *ws,
                    size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ L2 loss
 * Projection-domain loss of a batch of V views (the batch mean of Eq. 12 with
 * an L2 data term, Eq. 1):
 *   loss = (1/V) sum (proj - target)^2,   g_proj = 2 (proj - target) / V.
 * npix = nu * nv.  loss: device scalar.  g_proj may be NULL.
 * Needs the workspace from pmf_l2_loss_workspace(). */
size_t pmf_l2_loss_workspace(int64_t npix, int V);
int pmf_l2_loss(const float *proj, const float *target, int64_t npix, int V, float *loss,
                float *g_proj, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------- FDK initialisation
 * FDK reconstruction (Feldkamp et al. 1984) of the motion-averaged CBCT the
 * Gaussians are initialised from (Sec. 2.3.2): proj [V][nv][nu] measured
 * over a full circle (angles evenly covering 360 degrees; dtheta = 2 pi / V)
 * in pmf_project's geometry -> vol on grid (overwritten).  Cosine weighting,
 * ramp filtering of each detector row with the discrete Ram-Lak kernel of
 * the virtual pitch du SAD / SDD (rows zero-padded), then the voxel-driven
 * back-projection 1/2 sum dtheta (SAD / U)^2 q(a', b') with bilinear
 * interpolation between pixel centres (0 off the detector).  Errors:
 * PMF_EINVAL for null pointers, V outside [1, 65535], a bad grid or cone
 * (the volume must lie inside the source circle); PMF_EUNSUPPORTED for rows
 * longer than 4096 pixels, more than 65535 rows or (nu + 2)(nv + 2) >=
 * 2^27; PMF_EWORKSPACE if the workspace from pmf_fdk_workspace() is missing
 * or short.  The workspace holds mainly the filtered views, as zero-bordered
 * planes of 2 x 2 bilinear taps: 16 (nu + 2)(nv + 2) bytes per view. */
size_t pmf_fdk_workspace(const pmf_cone_t *cone, int V);
int pmf_fdk(const float *proj, const pmf_cone_t *cone, const float *angles, int V,
            const pmf_grid_t *grid, float *vol, void *ws, size_t ws_bytes, void *stream);

/* Grid-based sampling of a (FDK) volume into the initial reference Gaussians
 * (Sec. 2.3.2: sampled points keep their positions and the volume's
 * intensities as densities).  M = m[0] m[1] m[2] points on the lattice that
 * evenly fills the volume box: point (k0, k1, k2) at box_lo + (k + 1/2)
 * box_len / m per axis, axis 2 fastest; its density is the trilinear value
 * of vol there (the interpolation of pmf_warp); scale = `scale` on every
 * axis, quaternion (1, 0, 0, 0).  vol on grid (device, read); outputs
 * (device, written): mean [M][3], scale_out [M][3], quat [M][4], value
 * [M][1] -- a pmf_gauss_t with c = 1.  Errors: PMF_EINVAL for null
 * pointers, a bad grid, m[a] outside [1, n[a]] or scale not > 0.  No
 * workspace. */
int pmf_grid_init(const float *vol, const pmf_grid_t *grid, const int m[3], float scale,
                  float *mean, float *scale_out, float *quat, float *value, void *stream);

/* ------------------------------------------------- Stage 1 rasterizer
 * X-ray Gaussian splatting (Sec. 2.2, Eq. 7-9): per view each Gaussian of g
 * (c must be 1: its density rho) is mapped by the local affine approximation
 * of the cone-beam projection (Eq. 8; geometry of pmf_project: source at
 * SAD (cos th, sin th, 0), flat detector at SDD, pixel centres as for the
 * ray march) to a 2-D Gaussian with centre phi(p), covariance Sigma^ (the
 * projected Sigma~ = J W Sigma W^T J^T without its ray row and column) and
 * amplitude rho sqrt(2 pi |Sigma~| / |Sigma^|) (Eq. 9); each pixel of proj
 * [V][nv][nu] (overwritten) is the sum of these at its centre, each cut to
 * its ellipse (x - mu)^T Sigma^-1 (x - mu) <= trunc_k^2 (INFINITY: uncut;
 * every Gaussian then covers the whole detector).  Gaussians not in front of
 * the source are skipped.  Pixel sums are 32-bit fixed point with a per-tile
 * scale (each term exact to 2^-31 of the sum of the amplitudes that reach the
 * tile), so images repeat bit for bit.
 * pmf_rasterize_bwd overwrites grad (shapes of g) with the gradients of
 * sum(g_proj * proj), summed over the V views in order (the mask is not
 * differentiated); its sums run in a fixed order (the gradients repeat bit
 * for bit).  The workspace holds about 570 bytes per (Gaussian, view):
 * per-splat records, tile lists and per-tile partial gradients.  Errors: PMF_EINVAL for null pointers, c != 1, V < 1,
 * trunc_k <= 0 or a bad cone (0 < SAD < SDD, du, dv > 0, finite offsets);
 * PMF_EUNSUPPORTED for m * V >= 2^27 or detectors wider than 65536;
 * PMF_EWORKSPACE if the workspace from pmf_rasterize_workspace() is missing
 * or short.  m = 0 writes zeros. */
size_t pmf_rasterize_workspace(int64_t m, const pmf_cone_t *cone, int V);
int pmf_rasterize(const pmf_gauss_t *g, const pmf_cone_t *cone, const float *angles, int V,
                  float trunc_k, float *proj, void *ws, size_t ws_bytes, void *stream);
int pmf_rasterize_bwd(const pmf_gauss_t *g, const pmf_cone_t *cone, const float *angles, int V,
                      float trunc_k, const float *g_proj, const pmf_gauss_grad_t *grad, void *ws,
                      size_t ws_bytes, void *stream);
/* pmf_rasterize_bwd without its own binning: ws must be the workspace that a
 * pmf_rasterize call with the same g (unchanged), cone, angles, V and
 * trunc_k filled, on the same stream, with nothing else written to it since
 * (the splat records, tile lists and list positions are reused, as a
 * training step's forward and adjoint share them).  Same results, errors and
 * workspace size as pmf_rasterize_bwd; a workspace from anything else gives
 * wrong gradients (unchecked). */
int pmf_rasterize_bwd_binned(const pmf_gauss_t *g, const pmf_cone_t *cone, const float *angles,
                             int V, float trunc_k, const float *g_proj,
                             const pmf_gauss_grad_t *grad, void *ws, size_t ws_bytes,
                             void *stream);

/* ------------------------------------------------- Stage 2/3 loss terms
 * The loss terms that surround the motion path in Stages 2 and 3 (Sec.
 * 2.3.2, Eq. 10-14).  The paper leaves their discretisation open; the
 * readings taken are stated with each call.  All reductions are fixed-order
 * trees (deterministic).  Device pointers, caller-owned; loss is a device
 * scalar; stream-ordered, returns at once. */

/* L1 + D-SSIM projection loss of a batch of V views (Eq. 10 per view, batch
 * mean of Eq. 12), proj and target [V][nv][nu] (u fastest):
 *   loss = (1/V) sum_v [ mean |proj - target| + lambda_ssim (1 - SSIM_v) ],
 * SSIM_v the pixel mean of the SSIM map of Zhou et al. (2004): local means,
 * variances and covariance under an 11 x 11 Gaussian window (sigma 1.5,
 * normalised), zero padding outside the detector, C1 = 1e-4, C2 = 9e-4
 * (unit dynamic range); the paper sets lambda_ssim = 0.25.  g_proj (may be
 * NULL) is overwritten with d loss / d proj (d|r|/dr = 0 at r = 0).  Errors:
 * PMF_EINVAL for sizes < 1, a negative or non-finite lambda_ssim or a null
 * proj/target/loss; PMF_EWORKSPACE if the workspace from
 * pmf_l1_dssim_loss_workspace() is missing or short. */
size_t pmf_l1_dssim_loss_workspace(int nu, int nv, int V);
int pmf_l1_dssim_loss(const float *proj, const float *target, int nu, int nv, int V,
                      float lambda_ssim, float *loss, float *g_proj, void *ws, size_t ws_bytes,
                      void *stream);

/* Total variation of the D x D x D block of vol (on grid, axis 2 fastest)
 * whose first voxel is corner[3] (host array; Eq. 11, D = 32 and weight
 * lambda_tv = 0.05 in the paper; the block stands for the sub-volume
 * voxelized from the reference Gaussians):
 *   loss = weight / D^3 * sum over forward differences with both voxels in
 *          the block of |vol(p + e_a) - vol(p)|  (anisotropic TV),
 * and g_vol (may be NULL; same grid as vol) ACCUMULATES weight * d(TV)/d vol
 * on the block (d|r|/dr = 0 at r = 0), so the term adds onto the gradient
 * of the reference volume from the motion path.  Errors: PMF_EINVAL for a
 * bad grid, D < 1, a block outside the grid, a non-finite weight or null
 * vol/loss/corner; PMF_EWORKSPACE as above (pmf_tv_loss_workspace()). */
size_t pmf_tv_loss_workspace(int D);
int pmf_tv_loss(const float *vol, const pmf_grid_t *grid, const int32_t *corner, int D,
                float weight, float *loss, float *g_vol, void *ws, size_t ws_bytes, void *stream);

/* MBC normality loss (Eq. 13, weight lambda_MBC = 1 in Eq. 14) over the
 * basis volumes of L levels, bases[l] [C][n_l] on lvl[l] (C = 3 B channels
 * per level):
 *   loss = weight / (L C) * sum_{l,c} ( |E_l[c]|^2 - 1 )^2,
 * |E|^2 the sum of squares of the channel over its level's voxels (Eq. 13's
 * 1/9 is 1/(L C) for L = 3, B = 1).  g_bases (may be NULL; else L non-null
 * pointers with the shapes of bases) ACCUMULATES weight * d loss / d E, onto
 * the gradients of the bases from the motion path.  Errors: PMF_EINVAL for
 * L or C < 1, null pointers or bad grids, PMF_EUNSUPPORTED for L > 4;
 * PMF_EWORKSPACE as above (pmf_mbc_normality_loss_workspace()). */
/* pmf_tv_loss for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, checks, results (bit for bit) and accumulation into g_vol,
 * without a workspace.  Its per-block partial sums live in a static device
 * array of the library, one per GPU (32 KiB, held until the process ends),
 * sized for D <= PMF_TV_NOALLOC_MAX_D: a larger D returns PMF_EUNSUPPORTED
 * before anything is enqueued.  The call allocates nothing (no hipMalloc, no
 * library allocation); the first call on a device looks up that device's
 * copy of the array.  Every partial is written before it is read, so nothing
 * carries over between calls, but all calls on one GPU share the array:
 * calls that may overlap on one GPU (different streams, or threads without
 * ordering) race and must be serialised by the caller. */
#define PMF_TV_NOALLOC_MAX_D 128
int pmf_tv_loss_noalloc(const float *vol, const pmf_grid_t *grid, const int32_t *corner, int D,
                        float weight, float *loss, float *g_vol, void *stream);

size_t pmf_mbc_normality_loss_workspace(int L, int C);
int pmf_mbc_normality_loss(int L, int C, const float *const *bases, const pmf_grid_t *lvl,
                           float weight, float *loss, float *const *g_bases, void *ws,
                           size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ utility
 * dst[i] += src[i] for i < n: accumulation of per-view gradients by callers
 * that run the steps one view at a time. */
int pmf_accumulate(float *dst, const float *src, int64_t n, void *stream);

/* dst[i] = value for i < n, by a fill kernel (never a memset node, so it may
 * be recorded into a graph): buffers that gradients accumulate into. */
int pmf_fill(float *dst, int64_t n, float value, void *stream);

/* ---------------------------------------------------------- profiling
 * Per-kernel GPU time for measurement.  While enabled, every kernel launch
 * of the library is bracketed by two HIP events recorded on the stream it
 * is launched on.  pmf_profile returns the previous state.  pmf_profile_read
 * waits for, sums and discards the records of one kernel name (total_ms over
 * count launches).  pmf_profile_names writes the comma-separated names that
 * hold records into buf (host, len bytes, NUL-terminated) and returns the
 * full length.  Not for use while a stream is being captured into a graph. */
int pmf_profile(int enable);
int pmf_profile_read(const char *kernel, double *total_ms, int64_t *count);
size_t pmf_profile_names(char *buf, size_t len);

/* ------------------------------------------------------- launch shapes
 * Tunable launch shapes (process-wide; results do not depend on them beyond
 * float summation order).  Knobs:
 *   PMF_TUNE_PROJECT_TILE      ray tile of the forward projection: the pixels
 *                              one wavefront marches (u x v) and the
 *                              workgroup's tile: 0 = 16x4 in 16x16,
 *                              1 = 8x8 in 16x16, 2 = 4x16 in 16x16,
 *                              3 = 2x32 in 8x32, 4 = 32x2 in 32x8,
 *                              5 = 1x64 in 4x64 (default), 6 = 2x32 in 4x64,
 *                              7 = 1x64 in 2x128, 8 = 2x32 in 2x128;
 *   PMF_TUNE_BACKPROJECT_BRICK cell brick of the adjoint projection, L x W x H
 *                              (L along the horizontal axis a view's rays
 *                              mostly follow, H along z), 8 wavefronts unless
 *                              noted, with
 *                              consecutive samples of a ray in one cell
 *                              summed in registers first unless noted:
 *                              0 = 48x16x8 and 1 = 48x16x8 summing each
 *                              sample alone, one brick per workgroup; the
 *                              others walked in chunks of 8 bricks along z
 *                              by one workgroup: 2 = 32x16x8, 3 = 44x16x8,
 *                              4 (default) = 44x20x8, 5 = 40x20x8,
 *                              6 = 48x16x8, 7 = 64x16x8 with 12
 *                              wavefronts, 8 = 52x16x8 (a launch of few
 *                              views takes shorter chunks, so that it still
 *                              fills the chip);
 *   PMF_TUNE_VOXELIZE_BWD      Gaussians per wavefront in pmf_voxelize_bwd:
 *                              0 = chosen from the set's size (default),
 *                              k = 1..7: 2^(k-1).
 * pmf_tune_candidates returns the number of choices of a knob (0 for an
 * unknown knob); pmf_tune_set returns the previous choice or PMF_EINVAL for an
 * unknown knob or a choice out of range; pmf_tune_get returns the current
 * choice.  Not to be changed while another thread launches library work. */
enum { PMF_TUNE_PROJECT_TILE = 0, PMF_TUNE_BACKPROJECT_BRICK = 1, PMF_TUNE_VOXELIZE_BWD = 2 };
int pmf_tune_candidates(int knob);
int pmf_tune_get(int knob);
int pmf_tune_set(int knob, int choice);

/* Autotuner of the projection launch shapes: times every candidate of
 * PMF_TUNE_PROJECT_TILE with pmf_project and every candidate of
 * PMF_TUNE_BACKPROJECT_BRICK with pmf_project_bwd (per-view volumes) on the
 * caller's buffers, one warm-up and `reps` timed launches each (HIP events on
 * `stream`), and keeps the fastest of each knob.  vol [V][N] and g_proj
 * [V][nv][nu] are read; proj [V][nv][nu] and g_vol [V][N] are overwritten
 * (scratch); ws is the pmf_project_bwd workspace.  ms (host, optional)
 * receives the mean time per launch of each candidate, the projection tiles
 * first, then the bricks.  Synchronises the stream; returns PMF_OK or an
 * error (the previous choices are then restored). */
int pmf_autotune_project(const float *vol, const pmf_grid_t *grid, const pmf_cone_t *cone,
                         const float *angles, int V, float *proj, const float *g_proj,
                         float *g_vol, void *ws, size_t ws_bytes, int reps, float *ms,
                         void *stream);

/* Autotuner with a persistent cache of the chosen shapes: as
 * pmf_autotune_project, but first looks up cache_path (a text file of
 * "key<TAB>tile<TAB>brick" lines, key = the device's architecture, name and
 * compute-unit count, the grid, the cone geometry and V).  A hit sets both
 * knobs without timing anything (*cached = 1; ms is not written); a miss
 * times every candidate as pmf_autotune_project does and appends the choice
 * (*cached = 0).  cache_path NULL: no cache.  cached may be NULL.  Errors as
 * pmf_autotune_project, plus PMF_EINVAL if the cache cannot be written (the
 * tuned choice is then still set).  The views' cost is independent, so one
 * entry serves any draw of V views of the same scan geometry. */
int pmf_autotune(const char *cache_path, const float *vol, const pmf_grid_t *grid,
                 const pmf_cone_t *cone, const float *angles, int V, float *proj,
                 const float *g_proj, float *g_vol, void *ws, size_t ws_bytes, int reps, float *ms,
                 int *cached, void *stream);

/* ------------------------------------------------------- graph capture
 * A training step is a fixed sequence of launches over fixed buffers, so it
 * can be recorded once and replayed (the batched, many-view form of Sec. 4's
 * parallel DRRs, without a launch per kernel).  pmf_graph_capture records
 * everything record(user, stream) enqueues on `stream` (a non-null stream;
 * work forked to other streams must join it again before record returns)
 * into a HIP graph and instantiates it.  record returns PMF_OK or an error,
 * which pmf_graph_capture passes on (nothing is kept).  The recorded calls
 * must not allocate device memory: every buffer, workspace included, must
 * exist before capture and outlive the graph; a replay reads and writes the
 * same device addresses, so new inputs are copied into those buffers between
 * replays.  Profiling (pmf_profile) is off during the recording.  Library
 * calls clear memory with fill kernels, never with memset nodes; a recording
 * that holds a memset node is refused (PMF_EUNSUPPORTED).  pmf_graph_replay
 * launches the graph on `stream` (stream-ordered, returns at once);
 * pmf_graph_kernel_count gives the number of kernel nodes (-1 for NULL);
 * pmf_graph_destroy frees it (NULL: nothing to do).  A graph may be replayed
 * on one stream at a time. */
typedef struct pmf_graph pmf_graph_t;
typedef int (*pmf_record_fn)(void *user, void *stream);
int pmf_graph_capture(void *stream, pmf_record_fn record, void *user, pmf_graph_t **graph);
int pmf_graph_replay(const pmf_graph_t *graph, void *stream);
int64_t pmf_graph_kernel_count(const pmf_graph_t *graph);
int pmf_graph_destroy(pmf_graph_t *graph);

/* ----------------------------------------- batched motion path (fused)
 * All V views of the motion path in one pass over the bases:
 *   proj[v] = P_v( warp(ref, combine(bases, coeff[v])) )
 * i.e. the DVF of Eq. 3 from the MBC bases (Sec. 2.3.1) and the view's
 * coefficients, the pull-back warp of Eq. 2, and the line integrals of
 * Eq. 6, for every sampled view of a training iteration (Sec. 2.3.2).  The
 * DVFs are never written to memory; the warped volumes of all views live in
 * the workspace.  Arguments as in the calls above.  Needs the workspace from
 * pmf_warp_project_workspace(). */
size_t pmf_warp_project_workspace(int L, int B, const pmf_grid_t *lvl, int V,
                                    const pmf_grid_t *grid, const pmf_cone_t *cone);
int pmf_warp_project(const float *ref, const pmf_grid_t *grid, int L, int B,
                       const float *const *bases, const pmf_grid_t *lvl, const float *coeff,
                       int V, const pmf_cone_t *cone, const float *angles, float *proj,
                       void *ws, size_t ws_bytes, void *stream);

/* Adjoint of pmf_warp_project given g_proj [V][nv][nu] (the exact
 * transpose of the discrete Eq. 6, Eq. 2 and Eq. 3 chain, which the
 * training's gradient step through the forward model needs): writes g_ref
 * [N], g_bases (HOST array of L device pointers, [3B][N_l] each) and g_coeff
 * [V][L][B][3].  Recomputes every view's DVF instead of storing it; the
 * sums do not depend on scheduling (fixed point and fixed orders), so a call
 * repeats bit for bit.  Needs the workspace from
 * pmf_warp_project_bwd_workspace(). */
size_t pmf_warp_project_bwd_workspace(int L, int B, const pmf_grid_t *lvl, int V,
                                        const pmf_grid_t *grid, const pmf_cone_t *cone);
int pmf_warp_project_bwd(const float *ref, const pmf_grid_t *grid, int L, int B,
                           const float *const *bases, const pmf_grid_t *lvl, const float *coeff,
                           int V, const pmf_cone_t *cone, const float *angles,
                           const float *g_proj, float *g_ref, float *const *g_bases,
                           float *g_coeff, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------ ragged batch of scans
 * Up to PMF_MAX_SCANS independent scans (each its own reference volume,
 * grids, geometry and views; one motion model shape L, B for all) through
 * the motion path together: each stage is one kernel launch over the items
 * (voxels, detector tiles, bricks) of every scan, so small scans do not leave
 * the GPU idle and the whole batch is a handful of launches (the batched form
 * of the motion path extended to several instances; the views of a scan are
 * independent as in Sec. 2.3.2).
 *
 * pmf_scan_t describes one scan; all pointers are device pointers except
 * that the struct itself lives on the host.  Fields used by the forward call:
 * ref, grid, bases[0..L-1], lvl[0..L-1], coeff, V, cone, angles, proj.  The
 * adjoint call also reads g_proj and writes g_ref, g_bases[0..L-1], g_coeff
 * (layouts as in pmf_warp_project / pmf_warp_project_bwd).  Results equal
 * n_scans separate calls of pmf_warp_project / pmf_warp_project_bwd.
 * Workspaces are the sums of the per-scan workspaces; errors name the scan. */
#define PMF_MAX_SCANS 4
#define PMF_MAX_LEVELS 4
typedef struct {
    const float *ref;
    pmf_grid_t grid;
    const float *bases[PMF_MAX_LEVELS];
    pmf_grid_t lvl[PMF_MAX_LEVELS];
    const float *coeff;
    int32_t V;
    pmf_cone_t cone;
    const float *angles;
    float *proj;
    const float *g_proj;
    float *g_ref;
    float *g_bases[PMF_MAX_LEVELS];
    float *g_coeff;
} pmf_scan_t;

size_t pmf_warp_project_scans_workspace(int L, int B, const pmf_scan_t *scans, int n_scans);
int pmf_warp_project_scans(int L, int B, const pmf_scan_t *scans, int n_scans, void *ws,
                           size_t ws_bytes, void *stream);
size_t pmf_warp_project_bwd_scans_workspace(int L, int B, const pmf_scan_t *scans, int n_scans);
int pmf_warp_project_bwd_scans(int L, int B, const pmf_scan_t *scans, int n_scans, void *ws,
                               size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PMF_H */
