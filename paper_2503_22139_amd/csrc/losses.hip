// losses.hip -- the Stage 2/3 loss terms around the motion path (Sec. 2.3.2):
// the L1 + D-SSIM projection loss (Eq. 10, batch mean of Eq. 12), the
// total variation of a D^3 sub-volume of the reference volume (Eq. 11) and
// the MBC normality loss (Eq. 13), each with its gradient.
//
// Readings of the paper's unstated discretisations: L1 is the pixel mean of
// |x - y|; D-SSIM is 1 - SSIM with SSIM the pixel mean of the map of Zhou et
// al. (2004) under an 11 x 11 Gaussian window (sigma 1.5), zero padding
// outside the detector, C1 = 0.01^2, C2 = 0.03^2; TV is the anisotropic sum
// of |forward differences| inside the sub-volume over D^3; |e|^2 of Eq. 13
// is the sum of squares of a basis channel over its level grid, averaged over
// the L * C channels.  Subgradients of |.| at 0 are 0.  Every reduction is a
// fixed-order tree, so results are deterministic.
#include <algorithm>
#include <math.h>
#include <mutex>

#include "pmf_internal.h"

namespace pmf {

// ------------------------------------------------------------ L1 + D-SSIM
constexpr int SS_R = 5;                 // window radius (11 taps)
constexpr int SS_TU = 32, SS_TV = 16;   // output tile (u x v), one pixel per thread
constexpr int SS_HU = SS_TU + 2 * SS_R, SS_HV = SS_TV + 2 * SS_R;
constexpr int SS_THREADS = SS_TU * SS_TV;
constexpr float SS_C1 = 1e-4f, SS_C2 = 9e-4f;
constexpr int SS_NMAP = 5;              // dS/dmu_x, dS/dvar_x, dS/dcov, mu_x, mu_y

struct SsimW {
    float w[2 * SS_R + 1];
};

static SsimW ssim_window() {
    SsimW W;
    double s = 0.0, t[2 * SS_R + 1];
    for (int k = -SS_R; k <= SS_R; ++k) s += (t[k + SS_R] = exp(-0.5 * k * k / (1.5 * 1.5)));
    for (int k = 0; k <= 2 * SS_R; ++k) W.w[k] = (float)(t[k] / s);
    return W;
}

__device__ __forceinline__ float block_sum_512(float v, float *red) {
    v = wave_sum_lane63(v);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0)
        s = ((red[0] + red[1]) + (red[2] + red[3])) + ((red[4] + red[5]) + (red[6] + red[7]));
    return s;
}

// Per tile: the five local moments under the window (separable, in LDS),
// then per pixel the SSIM value and its partial derivatives with respect to
// the local mean, variance and covariance of x (written for the adjoint),
// and the tile's sums of SSIM and of |x - y|.  The window sums and the SSIM
// algebra run in double: variances are differences of second moments that
// cancel in float wherever the image is flat at a high level, and the
// constants C1, C2 are small against such levels (the double work is a few
// hundred operations per pixel).
__global__ __launch_bounds__(SS_THREADS) void k_ssim_fwd(const float *__restrict__ x,
                                                         const float *__restrict__ y, int nu,
                                                         int nv, int tiles_u, SsimW W,
                                                         float *__restrict__ maps, int64_t mstride,
                                                         float *__restrict__ partial) {
    __shared__ float sx[SS_HV][SS_HU], sy[SS_HV][SS_HU];
    __shared__ double hs[5][SS_HV][SS_TU];
    __shared__ float red[8];
    const int v = blockIdx.y, tile = blockIdx.x;
    const int u0 = (tile % tiles_u) * SS_TU, v0 = (tile / tiles_u) * SS_TV;
    const int64_t npix = (int64_t)nu * nv, base = (int64_t)v * npix;
    for (int i = threadIdx.x; i < SS_HV * SS_HU; i += SS_THREADS) {
        const int r = i / SS_HU, c = i - r * SS_HU;
        const int gu = u0 - SS_R + c, gv = v0 - SS_R + r;
        const bool in = gu >= 0 && gu < nu && gv >= 0 && gv < nv;
        const int64_t j = base + (int64_t)gv * nu + gu;
        sx[r][c] = in ? x[j] : 0.0f;
        sy[r][c] = in ? y[j] : 0.0f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SS_HV * SS_TU; i += SS_THREADS) {
        const int r = i / SS_TU, c = i - r * SS_TU;
        double a = 0.0, b = 0.0, aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
        for (int k = 0; k <= 2 * SS_R; ++k) {
            const double xv = sx[r][c + k], yv = sy[r][c + k], w = W.w[k];
            a = fma(w, xv, a);
            b = fma(w, yv, b);
            aa = fma(w * xv, xv, aa);
            bb = fma(w * yv, yv, bb);
            ab = fma(w * xv, yv, ab);
        }
        hs[0][r][c] = a;
        hs[1][r][c] = b;
        hs[2][r][c] = aa;
        hs[3][r][c] = bb;
        hs[4][r][c] = ab;
    }
    __syncthreads();
    const int r = threadIdx.x / SS_TU, c = threadIdx.x - r * SS_TU;
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k <= 2 * SS_R; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q) m[q] = fma((double)W.w[k], hs[q][r + k][c], m[q]);
    const int gu = u0 + c, gv = v0 + r;
    float s = 0.0f, ad = 0.0f;
    if (gu < nu && gv < nv) {
        const int64_t j = base + (int64_t)gv * nu + gu;
        const double mx = m[0], my = m[1];
        const double vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
        const double a1 = 2.0 * mx * my + SS_C1, a2 = 2.0 * cxy + SS_C2;
        const double b1 = mx * mx + my * my + SS_C1, b2 = vx + vy + SS_C2;
        const double inv = 1.0 / (b1 * b2);
        const double sd = a1 * a2 * inv;
        s = (float)sd;
        maps[j] = (float)(2.0 * my * a2 * inv - 2.0 * mx * sd / b1);   // dS/dmu_x
        maps[mstride + j] = (float)(-sd / b2);                         // dS/dvar_x
        maps[2 * mstride + j] = (float)(2.0 * a1 * inv);               // dS/dcov
        maps[3 * mstride + j] = (float)mx;
        maps[4 * mstride + j] = (float)my;
        ad = fabsf(x[j] - y[j]);
    }
    const float ts = block_sum_512(s, red);
    __syncthreads();
    const float ta = block_sum_512(ad, red);
    if (threadIdx.x == 0) {
        const int64_t t = (int64_t)v * gridDim.x + tile;
        partial[2 * t] = ta;
        partial[2 * t + 1] = ts;
    }
}

// Adjoint: dSSIM_sum/dx(i) = sum over pixels p in i's window of w(p - i) *
// [dS/dmu(p) + 2 (x(i) - mu_x(p)) dS/dvar(p) + (y(i) - mu_y(p)) dS/dcov(p)]
// = W*(dS/dmu - 2 mu_x dS/dvar - mu_y dS/dcov)(i) + 2 x(i) W*(dS/dvar)(i)
//   + y(i) W*(dS/dcov)(i), three separable window sums (the window is
// symmetric, zero outside), in double like the forward.
__global__ __launch_bounds__(SS_THREADS) void k_ssim_bwd(const float *__restrict__ x,
                                                         const float *__restrict__ y, int nu,
                                                         int nv, int tiles_u, SsimW W,
                                                         const float *__restrict__ maps,
                                                         int64_t mstride, float lam, float gscale,
                                                         float *__restrict__ g) {
    __shared__ double sm[3][SS_HV][SS_HU];
    __shared__ double hb[3][SS_HV][SS_TU];
    const int v = blockIdx.y, tile = blockIdx.x;
    const int u0 = (tile % tiles_u) * SS_TU, v0 = (tile / tiles_u) * SS_TV;
    const int64_t npix = (int64_t)nu * nv, base = (int64_t)v * npix;
    for (int i = threadIdx.x; i < SS_HV * SS_HU; i += SS_THREADS) {
        const int r = i / SS_HU, c = i - r * SS_HU;
        const int gu = u0 - SS_R + c, gv = v0 - SS_R + r;
        double p = 0.0, q = 0.0, t = 0.0;
        if (gu >= 0 && gu < nu && gv >= 0 && gv < nv) {
            const int64_t j = base + (int64_t)gv * nu + gu;
            q = maps[mstride + j];
            t = maps[2 * mstride + j];
            p = (double)maps[j] - 2.0 * (double)maps[3 * mstride + j] * q -
                (double)maps[4 * mstride + j] * t;
        }
        sm[0][r][c] = p;
        sm[1][r][c] = q;
        sm[2][r][c] = t;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SS_HV * SS_TU; i += SS_THREADS) {
        const int r = i / SS_TU, c = i - r * SS_TU;
        double a = 0.0, b = 0.0, e = 0.0;
#pragma unroll
        for (int k = 0; k <= 2 * SS_R; ++k) {
            const double w = W.w[k];
            a = fma(w, sm[0][r][c + k], a);
            b = fma(w, sm[1][r][c + k], b);
            e = fma(w, sm[2][r][c + k], e);
        }
        hb[0][r][c] = a;
        hb[1][r][c] = b;
        hb[2][r][c] = e;
    }
    __syncthreads();
    const int r = threadIdx.x / SS_TU, c = threadIdx.x - r * SS_TU;
    const int gu = u0 + c, gv = v0 + r;
    if (gu >= nu || gv >= nv) return;
    double bp = 0.0, bq = 0.0, bt = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * SS_R; ++k) {
        const double w = W.w[k];
        bp = fma(w, hb[0][r + k][c], bp);
        bq = fma(w, hb[1][r + k][c], bq);
        bt = fma(w, hb[2][r + k][c], bt);
    }
    const int64_t j = base + (int64_t)gv * nu + gu;
    const float xv = x[j], yv = y[j], d = xv - yv;
    const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    const double ds = bp + 2.0 * (double)xv * bq + (double)yv * bt;
    g[j] = (float)(gscale * ((double)sg - (double)lam * ds));
}

// loss = (1/V) sum_v [ sum|x - y| / npix + lam (1 - sum S / npix) ]: one
// wave per view sums its tiles (lane-strided, then a fixed DPP tree), then
// one thread sums the views in order.
__global__ __launch_bounds__(256) void k_ssim_final(const float *__restrict__ partial, int V,
                                                    int ntiles, float inv_npix, float lam,
                                                    float *__restrict__ vterm,
                                                    float *__restrict__ loss) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int v = wave; v < V; v += 4) {
        float a = 0.0f, s = 0.0f;
        for (int t = lane; t < ntiles; t += 64) {
            a += partial[2 * ((int64_t)v * ntiles + t)];
            s += partial[2 * ((int64_t)v * ntiles + t) + 1];
        }
        a = wave_sum_lane63(a);
        s = wave_sum_lane63(s);
        if (lane == 63) vterm[v] = a * inv_npix + lam * (1.0f - s * inv_npix);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int v = 0; v < V; ++v) t += vterm[v];
        *loss = t / (float)V;
    }
}

static int ssim_tiles(int nu, int nv, int &tiles_u) {
    tiles_u = (nu + SS_TU - 1) / SS_TU;
    return tiles_u * ((nv + SS_TV - 1) / SS_TV);
}

size_t l1_dssim_workspace(int nu, int nv, int V) {
    int tu;
    const int nt = ssim_tiles(nu, nv, tu);
    return align256(sizeof(float) * SS_NMAP * (size_t)nu * nv * V) +
           align256(sizeof(float) * 2 * (size_t)nt * V) + align256(sizeof(float) * (size_t)V);
}

hipError_t launch_l1_dssim(const float *proj, const float *target, int nu, int nv, int V,
                           float lam, float *loss, float *g, void *ws, hipStream_t s) {
    int tu;
    const int nt = ssim_tiles(nu, nv, tu);
    const int64_t mstride = (int64_t)nu * nv * V;
    float *maps = (float *)ws;
    float *partial = (float *)((char *)ws + align256(sizeof(float) * SS_NMAP * (size_t)mstride));
    float *vterm = (float *)((char *)partial + align256(sizeof(float) * 2 * (size_t)nt * V));
    const SsimW W = ssim_window();
    const dim3 grid((unsigned)nt, (unsigned)V);
    {
        ProfScope prof_("ssim_fwd", s);
        k_ssim_fwd<<<grid, SS_THREADS, 0, s>>>(proj, target, nu, nv, tu, W, maps, mstride, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope prof_("ssim_final", s);
        k_ssim_final<<<1, 256, 0, s>>>(partial, V, nt, 1.0f / (float)((int64_t)nu * nv), lam, vterm,
                                       loss);
    }
    if ((e = hipGetLastError()) != hipSuccess || !g) return e;
    {
        ProfScope prof_("ssim_bwd", s);
        k_ssim_bwd<<<grid, SS_THREADS, 0, s>>>(proj, target, nu, nv, tu, W, maps, mstride, lam,
                                               1.0f / ((float)((int64_t)nu * nv) * (float)V), g);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ TV of a block
constexpr int TV_THREADS = 256;

// One thread per voxel p of the D^3 block: its forward differences inside the
// block (loss) and d/dV(p) of the sum of |differences| (gradient, added to
// g_vol at p scaled by weight / D^3; each voxel is written by one thread).
__global__ __launch_bounds__(TV_THREADS) void k_tv(const float *__restrict__ vol, int n1, int n2,
                                                   int c0, int c1, int c2, int D, float scale,
                                                   float *__restrict__ g,
                                                   float *__restrict__ partial) {
    __shared__ float red[4];
    const int64_t idx = (int64_t)blockIdx.x * TV_THREADS + threadIdx.x;
    float acc = 0.0f;
    if (idx < (int64_t)D * D * D) {
        const int p2 = (int)(idx % D), p1 = (int)((idx / D) % D), p0 = (int)(idx / ((int64_t)D * D));
        const int64_t s1 = n2, s0 = (int64_t)n1 * n2;
        const int64_t j = (c0 + p0) * s0 + (int64_t)(c1 + p1) * s1 + (c2 + p2);
        const float v0 = vol[j];
        const int p[3] = {p0, p1, p2};
        const int64_t st[3] = {s0, s1, 1};
        float gs = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (p[a] + 1 < D) {
                const float d = vol[j + st[a]] - v0;
                acc += fabsf(d);
                gs -= d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            }
            if (p[a] >= 1) {
                const float d = v0 - vol[j - st[a]];
                gs += d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            }
        }
        if (g) g[j] += scale * gs;
    }
    acc = wave_sum_lane63(acc);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(64) void k_sum_scaled(const float *__restrict__ partial, int n,
                                                   float scale, float *__restrict__ out) {
    const float s = wave_sum_partials(partial, n);
    if (threadIdx.x == 63) *out = scale * s;
}

static int tv_blocks(int D) { return (int)(((int64_t)D * D * D + TV_THREADS - 1) / TV_THREADS); }

size_t tv_workspace(int D) { return align256(sizeof(float) * (size_t)tv_blocks(D)); }

// The two launches of the TV term; every partial is written by its block
// before k_sum_scaled reads it, so the buffer needs no clearing.
static hipError_t tv_launches(const float *vol, const GridK &gk, const int corner[3], int D,
                              float weight, float *loss, float *g, float *partial, bool prof,
                              hipStream_t s) {
    const int nb = tv_blocks(D);
    const float scale = weight / ((float)D * (float)D * (float)D);
    {
        ProfScope prof_(prof ? "tv" : nullptr, s);
        k_tv<<<(unsigned)nb, TV_THREADS, 0, s>>>(vol, gk.n[1], gk.n[2], corner[0], corner[1],
                                                 corner[2], D, scale, g, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum_scaled<<<1, 64, 0, s>>>(partial, nb, scale, loss);
    return hipGetLastError();
}

hipError_t launch_tv(const float *vol, const GridK &gk, const int corner[3], int D, float weight,
                     float *loss, float *g, void *ws, hipStream_t s) {
    return tv_launches(vol, gk, corner, D, weight, loss, g, (float *)ws, true, s);
}

// Scratch of the allocation-free TV call: the per-block partial sums for
// blocks up to TV_NOALLOC_MAX_D^3 voxels, one copy per device for the life of
// the process.  Host code never passes `scratch` itself (on the host it names
// a stand-in, not device memory): tv_scratch_ptr looks up each device's
// address once and kernels receive that.
static __device__ __align__(256) float scratch[(TV_NOALLOC_MAX_D * TV_NOALLOC_MAX_D *
                                                    TV_NOALLOC_MAX_D + TV_THREADS - 1) /
                                                   TV_THREADS];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device, resolved on the first
// call made with that device current.
static hipError_t tv_scratch_ptr(float **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_tv_noalloc(const float *vol, const GridK &gk, const int corner[3], int D,
                             float weight, float *loss, float *g, hipStream_t s) {
    if (D < 1 || D > TV_NOALLOC_MAX_D) return hipErrorInvalidValue;
    float *partial = nullptr;
    hipError_t e = tv_scratch_ptr(&partial);
    if (e != hipSuccess) return e;
    return tv_launches(vol, gk, corner, D, weight, loss, g, partial, false, s);
}

// ------------------------------------------------------- MBC normality (Eq. 13)
constexpr int NRM_BLOCKS = 256;         // partial sums per channel

// Sum of squares of each channel of one level ([C][N]): NRM_BLOCKS fixed
// strided partials per channel.  VEC: the channels are 16-byte aligned and
// N % 4 == 0, and the values move as float4.
template <bool VEC>
__global__ __launch_bounds__(256) void k_sumsq(const float *__restrict__ e, int64_t N,
                                               float *__restrict__ partial) {
    __shared__ float red[4];
    const int ch = blockIdx.y;
    const float *ec = e + (int64_t)ch * N;
    float acc = 0.0f;
    if (VEC) {
        const float4 *e4 = (const float4 *)ec;
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N / 4;
             i += (int64_t)NRM_BLOCKS * 256) {
            const float4 x = e4[i];
            acc = fmaf(x.x, x.x, acc);
            acc = fmaf(x.y, x.y, acc);
            acc = fmaf(x.z, x.z, acc);
            acc = fmaf(x.w, x.w, acc);
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
             i += (int64_t)NRM_BLOCKS * 256)
            acc = fmaf(ec[i], ec[i], acc);
    }
    acc = wave_sum_lane63(acc);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[(int64_t)ch * NRM_BLOCKS + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Per channel |e|^2 (one wave per channel, fixed tree), the factor
// weight * 4 (|e|^2 - 1) / nch of its gradient, and
// loss = weight * sum (|e|^2 - 1)^2 / nch.
__global__ __launch_bounds__(256) void k_norm_final(const float *__restrict__ partial, int nch,
                                                    float weight, float *__restrict__ fac,
                                                    float *__restrict__ loss) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int ch = wave; ch < nch; ch += 4) {
        float s = 0.0f;
        for (int b = lane; b < NRM_BLOCKS; b += 64) s += partial[(int64_t)ch * NRM_BLOCKS + b];
        s = wave_sum_lane63(s);
        if (lane == 63) {
            fac[nch + ch] = (s - 1.0f) * (s - 1.0f);
            fac[ch] = weight * 4.0f * (s - 1.0f) / (float)nch;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int ch = 0; ch < nch; ++ch) t += fac[nch + ch];
        *loss = weight * t / (float)nch;
    }
}

// g[c][j] += fac[c] * e[c][j]; grid (blocks per channel, C).  VEC as for
// k_sumsq (g aligned too).
template <bool VEC>
__global__ __launch_bounds__(256) void k_norm_grad(const float *__restrict__ e, int64_t N,
                                                   const float *__restrict__ fac,
                                                   float *__restrict__ g) {
    const int ch = blockIdx.y;
    const float f = fac[ch];
    const float *ec = e + (int64_t)ch * N;
    float *gc = g + (int64_t)ch * N;
    if (VEC) {
        const float4 *e4 = (const float4 *)ec;
        float4 *g4 = (float4 *)gc;
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N / 4;
             i += (int64_t)gridDim.x * 256) {
            const float4 x = e4[i];
            float4 y = g4[i];
            y.x = fmaf(f, x.x, y.x);
            y.y = fmaf(f, x.y, y.y);
            y.z = fmaf(f, x.z, y.z);
            y.w = fmaf(f, x.w, y.w);
            g4[i] = y;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
             i += (int64_t)gridDim.x * 256)
            gc[i] = fmaf(f, ec[i], gc[i]);
    }
}

size_t normality_workspace(int L, int C) {
    return align256(sizeof(float) * (size_t)L * C * NRM_BLOCKS) + align256(sizeof(float) * 2 * (size_t)L * C);
}

hipError_t launch_normality(int L, int C, const float *const *bases, const GridK *lg,
                            float weight, float *loss, float *const *g, void *ws, hipStream_t s) {
    float *partial = (float *)ws;
    float *fac = (float *)((char *)ws + align256(sizeof(float) * (size_t)L * C * NRM_BLOCKS));
    hipError_t e;
    for (int l = 0; l < L; ++l) {
        const int64_t N = grid_size(lg[l]);
        const bool vec = (N & 3) == 0 && ((uintptr_t)bases[l] & 15) == 0;
        {
            ProfScope prof_("normality", s);
            float *pl = partial + (int64_t)l * C * NRM_BLOCKS;
            if (vec)
                k_sumsq<true><<<dim3(NRM_BLOCKS, (unsigned)C), 256, 0, s>>>(bases[l], N, pl);
            else
                k_sumsq<false><<<dim3(NRM_BLOCKS, (unsigned)C), 256, 0, s>>>(bases[l], N, pl);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    k_norm_final<<<1, 256, 0, s>>>(partial, L * C, weight, fac, loss);
    if ((e = hipGetLastError()) != hipSuccess || !g) return e;
    for (int l = 0; l < L; ++l) {
        const int64_t N = grid_size(lg[l]);
        const bool vec = (N & 3) == 0 && (((uintptr_t)bases[l] | (uintptr_t)g[l]) & 15) == 0;
        const int64_t items = vec ? N / 4 : N;
        const int64_t blocks = std::min<int64_t>((items + 255) / 256, 1024);
        {
            ProfScope prof_("normality", s);
            if (vec)
                k_norm_grad<true><<<dim3((unsigned)blocks, (unsigned)C), 256, 0, s>>>(
                    bases[l], N, fac + (int64_t)l * C, g[l]);
            else
                k_norm_grad<false><<<dim3((unsigned)blocks, (unsigned)C), 256, 0, s>>>(
                    bases[l], N, fac + (int64_t)l * C, g[l]);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pmf
