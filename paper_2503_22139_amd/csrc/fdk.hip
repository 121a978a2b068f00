// fdk.hip -- FDK reconstruction (Feldkamp et al. 1984), the motion-averaged
// CBCT from which the Gaussians are initialised (Sec. 2.3.2).
//
// Circular orbit, flat detector, in the projector's geometry, written on the
// virtual detector through the isocentre (pitches scaled by SAD / SDD):
// cosine weighting SDD / sqrt(SDD^2 + a^2 + b^2); ramp filtering of each
// detector row with the discrete Ram-Lak kernel of the virtual pitch tau
// (h[0] = 1 / (4 tau^2), h[n odd] = -1 / (pi n tau)^2, rows zero-padded),
// q = tau (h * p~); voxel-driven back-projection f(x) = 1/2 sum_views
// dtheta (SAD / U)^2 q(a', b'), U the depth of x along the central ray,
// (a', b') = SAD (t_u, t_v) / U, bilinear between pixel centres (0 off the
// detector), dtheta = 2 pi / V.  The plain Ram-Lak kernel, linear
// interpolation and full-scan weighting 1/2 are the readings of the paper's
// "quick FDK reconstruction".
//
// Layout of the filtered projections (workspace): per view a zero-bordered
// plane of (nv + 2) x (nu + 2) float4 "quads"; quad (j, c) holds the four
// bilinear taps qp(j, c), qp(j, c + 1), qp(j + 1, c), qp(j + 1, c + 1) of the
// padded image qp(j, c) = q[j - 1][c - 1] (0 on the border and beyond).  A
// back-projection sample clamps its padded pixel coordinates into
// [0, nu + 1] x [0, nv + 1] -- any sample that leaves the detector then reads
// zero taps, exactly as the definition asks -- and fetches its whole 2 x 2
// neighbourhood with one 16-byte load, with no bounds test.
#include <math.h>

#include "pmf_internal.h"

namespace pmf {

constexpr int FDK_R = 8;               // outputs per lane per chunk: n = b0 + lane + 64 j
constexpr int FDK_CH = 64 * FDK_R;     // outputs per chunk
constexpr int FDK_PAD = 64;            // zeros on each side of the row in LDS
constexpr int BP_ZC = 16;              // voxels along axis 2 per back-projection thread

// First (odd) lag of the tap table and its number of rows.
static inline int fdk_t0(int nu) { return 1 - 2 * ((nu + 1) / 2); }
static inline int fdk_taps(int nu) {
    const int bmax = ((nu - 1) / FDK_CH) * FDK_CH;
    return (bmax + 63 - fdk_t0(nu)) / 2 + 1;
}

// Tap table of the odd lags: wt[k][j] = -1 / (pi^2 tau d^2), d = t0 + 2k +
// 64j -- the weight of input m for output n when n - m = d.  Uniform per
// loop step of the filter, so the filter reads eight of them with one
// scalar load.
__global__ void k_fdk_taps(double tau, int t0, int K, double *__restrict__ wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K * FDK_R) return;
    const double d = (double)t0 + 2.0 * (i / FDK_R) + 64.0 * (i % FDK_R);
    wt[i] = -1.0 / (M_PI * M_PI * tau * d * d);
}

// One wave per (detector row i, view v): cosine-weighted row into LDS (zero
// borders), the filtered row q[n] = p~[n] / (4 tau) + sum_{n - m odd}
// wt(n - m) p~[m] with each lane owning the outputs b0 + lane + 64 j (the
// lag n - m = t + 64 j then depends on the loop counter t and j only), then
// the row's taps written into the quads of padded rows i + 1 (top pair) and
// i (bottom pair).  Block row nv writes the plane's zero border rows.  The
// row and the sums are double: for smooth rows on fine pixels q is a small
// difference of the centre tap and the long odd-lag sum (they cancel exactly
// on a constant row), and float sums of ~nu/2 terms lose its low digits.
// On gfx950 a double FMA issues at the rate of an unpacked float one.
__global__ __launch_bounds__(64) void k_fdk_filter(const float *__restrict__ proj, pmf_cone_t c,
                                                   const double *__restrict__ wt, int t0,
                                                   float4 *__restrict__ qq) {
    extern __shared__ double lds[];
    const int nu = c.nu, nv = c.nv, lane = threadIdx.x;
    const int i = blockIdx.x, v = blockIdx.y;
    const int P = nu + 2;
    float4 *const plane = qq + (int64_t)v * (nv + 2) * P;
    float2 *const half = (float2 *)plane;           // quad e: half[2e] = top, half[2e + 1] = bottom
    if (i == nv) {
        for (int col = lane; col < P; col += 64) {
            half[2 * (int64_t)col] = make_float2(0.0f, 0.0f);
            half[2 * ((int64_t)nv * P + col) + 1] = make_float2(0.0f, 0.0f);
            plane[(int64_t)(nv + 1) * P + col] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        return;
    }
    double *const row = lds;                         // row[m + FDK_PAD], m in [-64, nu + 64)
    // out[n + 1] = q[n]; out[0] = out[nu + 1] = out[nu + 2] = 0 (the last
    // quad column pairs the border tap nu + 1 with the one beyond it)
    float *const out = (float *)(lds + nu + 2 * FDK_PAD);
    const int64_t base = ((int64_t)v * nv + i) * nu;
    const double b = ((double)i - 0.5 * (nv - 1) + c.off_v) * c.dv;
    const double sdd = c.sdd, sb = sdd * sdd + b * b;
    for (int m = lane - FDK_PAD; m < nu + FDK_PAD; m += 64) {
        double x = 0.0;
        if (m >= 0 && m < nu) {
            const double a = ((double)m - 0.5 * (nu - 1) + c.off_u) * c.du;
            x = (double)proj[base + m] * sdd / sqrt(sb + a * a);
        }
        row[m + FDK_PAD] = x;
    }
    if (lane == 0) {
        out[0] = 0.0f;
        out[nu + 1] = 0.0f;
        out[nu + 2] = 0.0f;
    }
    __syncthreads();
    const double c0 = (double)c.sdd / (4.0 * (double)c.du * c.sad);
    for (int b0 = 0; b0 < nu; b0 += FDK_CH) {
        double acc[FDK_R];
#pragma unroll
        for (int j = 0; j < FDK_R; ++j) acc[j] = 0.0;
        const int ts = (b0 - nu + 1) | 1;            // first odd lag with an input on the row
        const double *wk = wt + ((ts - t0) >> 1) * FDK_R;
        const double *xr = row + FDK_PAD + b0 + lane - ts;
#pragma unroll 4
        for (int t = ts; t <= b0 + 63; t += 2, wk += FDK_R, xr -= 2) {
            const double x = *xr;
#pragma unroll
            for (int j = 0; j < FDK_R; ++j) acc[j] = fma(wk[j], x, acc[j]);
        }
#pragma unroll
        for (int j = 0; j < FDK_R; ++j) {
            const int n = b0 + lane + 64 * j;
            if (n < nu) out[n + 1] = (float)fma(c0, row[FDK_PAD + n], acc[j]);
        }
    }
    __syncthreads();
    for (int col = lane; col < P; col += 64) {
        const float2 p = make_float2(out[col], out[col + 1]);
        half[2 * ((int64_t)(i + 1) * P + col)] = p;
        half[2 * ((int64_t)i * P + col) + 1] = p;
    }
}

struct FdkView {
    float ct, st, sx, sy;    // cos, sin, source position SAD (cos, sin)
};

__global__ void k_fdk_views(const float *__restrict__ angles, int V, float sad,
                            FdkView *__restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double th = angles[v], ct = cos(th), st = sin(th);
    out[v] = {(float)ct, (float)st, (float)(sad * ct), (float)(sad * st)};
}

struct FdkBp {
    float sad, inv_tu, inv_tv, cu, cv, umax, vmax, wsc, hz;
    unsigned row_bytes;      // (nu + 2) * 16
    int64_t plane_bytes;     // (nv + 2) * row_bytes
    int tx, ty;              // 16 x 16 column tiles along axes 0, 1
};

// Workgroup = 16 x 16 voxel columns (each wave an 8 x 8 patch, so one wave's
// samples of a view fall on a few neighbouring detector cache lines) x
// BP_ZC voxels along axis 2 per thread.  Per view the column's geometry
// (depth U, magnification, u coordinate) is computed once; along the column
// only v moves, linearly.  Views are summed in order.  Workgroups are
// numbered so that each XCD gets a contiguous slab along axis 2 (one band of
// detector rows in every view).  Threads past the grid edge compute on
// clamped positions and store nothing.
__global__ __launch_bounds__(256, 8) void k_fdk_bp(const float4 *__restrict__ qq, FdkBp p,
                                                const FdkView *__restrict__ views, int V, GridK g,
                                                float *__restrict__ vol) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int tiles = p.tx * p.ty;
    const int zc = b / tiles, tile = b - zc * tiles;
    const int tyi = tile / p.tx, txi = tile - tyi * p.tx;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ix = txi * 16 + (w & 1) * 8 + (lane & 7);
    const int iy = tyi * 16 + (w >> 1) * 8 + (lane >> 3);
    const int iz0 = zc * BP_ZC;
    const float x = g.c0[0] + min(ix, g.n[0] - 1) * g.h[0];
    const float y = g.c0[1] + min(iy, g.n[1] - 1) * g.h[1];
    const float z0 = g.c0[2] + iz0 * g.h[2];
    float acc[BP_ZC];
#pragma unroll
    for (int k = 0; k < BP_ZC; ++k) acc[k] = 0.0f;
    const char *pl = (const char *)qq;
    for (int v = 0; v < V; ++v, pl += p.plane_bytes) {
        const FdkView w = views[v];
        const float dx = x - w.sx, dy = y - w.sy;
        const float tu = fmaf(-w.st, dx, w.ct * dy);
        const float U = -fmaf(w.ct, dx, w.st * dy);
        const float r = p.sad / U;
        const float fu = __builtin_amdgcn_fmed3f(fmaf(r * tu, p.inv_tu, p.cu), 0.0f, p.umax);
        const float wu = __builtin_amdgcn_fractf(fu);
        const unsigned colb = (unsigned)(int)fu * 16u;
        const float wr2 = p.wsc * r * r;
        const float rv = r * p.inv_tv;
        const float fv0 = fmaf(rv, z0, p.cv), dfv = rv * p.hz;
#pragma unroll
        for (int k = 0; k < BP_ZC; ++k) {
            const float fv = __builtin_amdgcn_fmed3f(fmaf((float)k, dfv, fv0), 0.0f, p.vmax);
            const float wv = __builtin_amdgcn_fractf(fv);
            const unsigned off = __umul24((unsigned)(int)fv, p.row_bytes) + colb;
            const float4 e = *(const float4 *)(pl + off);
            const float top = fmaf(wu, e.y - e.x, e.x), bot = fmaf(wu, e.w - e.z, e.z);
            acc[k] = fmaf(wr2, fmaf(wv, bot - top, top), acc[k]);
        }
    }
    if (ix >= g.n[0] || iy >= g.n[1]) return;
    float *o = vol + ((int64_t)ix * g.n[1] + iy) * g.n[2];
#pragma unroll
    for (int k = 0; k < BP_ZC; ++k)
        if (iz0 + k < g.n[2]) o[iz0 + k] = acc[k];
}

static size_t fdk_plane_bytes(const pmf_cone_t &c) {
    return sizeof(float4) * (size_t)(c.nu + 2) * (c.nv + 2);
}

size_t fdk_workspace(const pmf_cone_t &c, int V) {
    return align256(fdk_plane_bytes(c) * V) + align256(sizeof(FdkView) * (size_t)V) +
           align256(sizeof(double) * FDK_R * (size_t)fdk_taps(c.nu));
}

size_t fdk_filter_lds(const pmf_cone_t &c) {
    return sizeof(double) * (size_t)(c.nu + 2 * FDK_PAD) + sizeof(float) * (size_t)(c.nu + 3);
}

hipError_t launch_fdk(const float *proj, const pmf_cone_t &c, const float *angles, int V,
                      const GridK &g, float *vol, void *ws, hipStream_t s) {
    char *w = (char *)ws;
    float4 *qq = (float4 *)w;
    w += align256(fdk_plane_bytes(c) * V);
    FdkView *views = (FdkView *)w;
    w += align256(sizeof(FdkView) * (size_t)V);
    double *wt = (double *)w;
    const double tau = (double)c.du * c.sad / c.sdd;
    const int t0 = fdk_t0(c.nu), K = fdk_taps(c.nu);
    hipError_t e;
    k_fdk_taps<<<(unsigned)((K * FDK_R + 255) / 256), 256, 0, s>>>(tau, t0, K, wt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_fdk_views<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(angles, V, c.sad, views);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        ProfScope prof_("fdk_filter", s);
        k_fdk_filter<<<dim3((unsigned)c.nv + 1, (unsigned)V), 64, fdk_filter_lds(c), s>>>(proj, c, wt,
                                                                                         t0, qq);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    FdkBp p;
    p.sad = c.sad;
    p.inv_tu = (float)((double)c.sdd / ((double)c.du * c.sad));
    p.inv_tv = (float)((double)c.sdd / ((double)c.dv * c.sad));
    p.cu = (float)(0.5 * (c.nu - 1) - c.off_u + 1.0);
    p.cv = (float)(0.5 * (c.nv - 1) - c.off_v + 1.0);
    p.umax = (float)(c.nu + 1);
    p.vmax = (float)(c.nv + 1);
    p.wsc = (float)(M_PI / V);
    p.hz = g.h[2];
    p.row_bytes = 16u * (unsigned)(c.nu + 2);
    p.plane_bytes = (int64_t)fdk_plane_bytes(c);
    p.tx = (g.n[0] + 15) / 16;
    p.ty = (g.n[1] + 15) / 16;
    const int64_t nb = (int64_t)p.tx * p.ty * ((g.n[2] + BP_ZC - 1) / BP_ZC);
    {
        ProfScope prof_("fdk_backproject", s);
        k_fdk_bp<<<(unsigned)nb, 256, 0, s>>>(qq, p, views, V, g, vol);
    }
    return hipGetLastError();
}

// Grid-based sampling of the FDK volume into initial Gaussians (Sec.
// 2.3.2): a lattice of m0 x m1 x m2 points evenly filling the volume box
// (point k at box_lo + (k + 1/2) box_len / m per axis, axis 2 fastest); each
// point keeps its position and the volume's trilinear value there as its
// density; isotropic scale s, identity rotation.
__global__ void k_grid_init(const float *__restrict__ vol, GridK g, int m0, int m1, int m2,
                            float s, float *__restrict__ mean, float *__restrict__ scale,
                            float *__restrict__ quat, float *__restrict__ value) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)m0 * m1 * m2) return;
    const int k2 = (int)(k % m2), k1 = (int)((k / m2) % m1), k0 = (int)(k / ((int64_t)m2 * m1));
    const int kk[3] = {k0, k1, k2}, mm[3] = {m0, m1, m2};
    float u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // voxel-unit coordinate of the point (voxel 0's centre at 0)
        const double ua = ((double)kk[a] + 0.5) * g.n[a] / mm[a] - 0.5;
        u[a] = (float)ua;
        mean[3 * k + a] = (float)(g.c0d[a] + ua * g.hd[a]);
        scale[3 * k + a] = s;
    }
    quat[4 * k + 0] = 1.0f;
    quat[4 * k + 1] = 0.0f;
    quat[4 * k + 2] = 0.0f;
    quat[4 * k + 3] = 0.0f;
    value[k] = sample_u(vol, g.n, u[0], u[1], u[2]);
}

hipError_t launch_grid_init(const float *vol, const GridK &g, const int m[3], float s,
                            float *mean, float *scale, float *quat, float *value, hipStream_t st) {
    const int64_t M = (int64_t)m[0] * m[1] * m[2];
    k_grid_init<<<(unsigned)((M + 255) / 256), 256, 0, st>>>(vol, g, m[0], m[1], m[2], s, mean,
                                                              scale, quat, value);
    return hipGetLastError();
}

}  // namespace pmf
