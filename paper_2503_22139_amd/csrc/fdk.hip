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
#include <math.h>

#include "pmf_internal.h"

namespace pmf {

constexpr int FDK_MAXU = 8192;          // detector row length held in LDS

// One workgroup per (row, view): the weighted row in LDS, then per output
// pixel n: q[n] = p~[n] / (4 tau) - 1 / (pi^2 tau) sum_{d odd} (p~[n-d] +
// p~[n+d]) / d^2.
__global__ __launch_bounds__(256) void k_fdk_filter(const float *__restrict__ proj, pmf_cone_t c,
                                                    float *__restrict__ q) {
    __shared__ float row[FDK_MAXU];
    __shared__ float inv_d2[FDK_MAXU / 2];
    const int iv = blockIdx.x, v = blockIdx.y, nu = c.nu;
    const int64_t base = ((int64_t)v * c.nv + iv) * nu;
    const double b = ((double)iv - 0.5 * (c.nv - 1) + c.off_v) * c.dv;
    const double sdd2 = (double)c.sdd * c.sdd;
    for (int i = threadIdx.x; i < nu; i += blockDim.x) {
        const double a = ((double)i - 0.5 * (nu - 1) + c.off_u) * c.du;
        row[i] = (float)((double)proj[base + i] * (double)c.sdd / sqrt(sdd2 + a * a + b * b));
    }
    for (int k = threadIdx.x; k < (nu + 1) / 2; k += blockDim.x) {
        const double d = 2.0 * k + 1.0;
        inv_d2[k] = (float)(1.0 / (d * d));
    }
    __syncthreads();
    const double tau = (double)c.du * c.sad / c.sdd;
    const float c0 = (float)(1.0 / (4.0 * tau)), c1 = (float)(1.0 / (M_PI * M_PI * tau));
    for (int n = threadIdx.x; n < nu; n += blockDim.x) {
        float s = 0.0f;
        for (int k = 0; 2 * k + 1 < nu; ++k) {
            const int d = 2 * k + 1;
            const float lo = n - d >= 0 ? row[n - d] : 0.0f;
            const float hi = n + d < nu ? row[n + d] : 0.0f;
            s = fmaf(lo + hi, inv_d2[k], s);
        }
        q[base + n] = fmaf(c0, row[n], -c1 * s);
    }
}

struct FdkView {
    float ct, st;
};

__global__ void k_fdk_views(const float *__restrict__ angles, int V, FdkView *__restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double th = angles[v];
    out[v].ct = (float)cos(th);
    out[v].st = (float)sin(th);
}

// One thread per voxel (axis 2 fastest), views in order.
__global__ __launch_bounds__(256) void k_fdk_bp(const float *__restrict__ q, pmf_cone_t c, int V,
                                                const FdkView *__restrict__ views, GridK g,
                                                float *__restrict__ vol) {
    const int64_t N = grid_size(g);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int iz = (int)(j % g.n[2]);
    const int iy = (int)((j / g.n[2]) % g.n[1]);
    const int ix = (int)(j / ((int64_t)g.n[2] * g.n[1]));
    const float x = g.c0[0] + ix * g.h[0], y = g.c0[1] + iy * g.h[1], z = g.c0[2] + iz * g.h[2];
    const float sad = c.sad;
    const float inv_tu = (float)((double)c.sdd / ((double)c.du * c.sad));
    const float inv_tv = (float)((double)c.sdd / ((double)c.dv * c.sad));
    const float cu = 0.5f * (c.nu - 1) - c.off_u, cv = 0.5f * (c.nv - 1) - c.off_v;
    const float wsc = (float)(0.5 * 2.0 * M_PI / V);
    float acc = 0.0f;
    for (int v = 0; v < V; ++v) {
        const FdkView w = views[v];
        const float dx = x - sad * w.ct, dy = y - sad * w.st;
        const float tu = -w.st * dx + w.ct * dy;
        const float U = -w.ct * dx - w.st * dy;
        const float r = sad / U;
        const float fu = r * tu * inv_tu + cu, fv = r * z * inv_tv + cv;
        const float f0 = floorf(fu), f1 = floorf(fv);
        const int i0 = (int)f0, k0 = (int)f1;
        const float wu = fu - f0, wv = fv - f1;
        const float *qv = q + (int64_t)v * c.nv * c.nu;
        float s = 0.0f;
#pragma unroll
        for (int dk = 0; dk < 2; ++dk) {
            const int kk = k0 + dk;
            if (kk < 0 || kk >= c.nv) continue;
            const float wk = dk ? wv : 1.0f - wv;
            const float *qr = qv + (int64_t)kk * c.nu;
            const float a = (i0 >= 0 && i0 < c.nu) ? qr[i0] : 0.0f;
            const float b = (i0 + 1 >= 0 && i0 + 1 < c.nu) ? qr[i0 + 1] : 0.0f;
            s = fmaf(wk, fmaf(wu, b - a, a), s);
        }
        acc = fmaf(wsc * r * r, s, acc);
    }
    vol[j] = acc;
}

size_t fdk_workspace(const pmf_cone_t &c, int V) {
    return align256(sizeof(float) * (size_t)c.nu * c.nv * V) + align256(sizeof(FdkView) * (size_t)V);
}

hipError_t launch_fdk(const float *proj, const pmf_cone_t &c, const float *angles, int V,
                      const GridK &g, float *vol, void *ws, hipStream_t s) {
    float *q = (float *)ws;
    FdkView *views = (FdkView *)((char *)ws + align256(sizeof(float) * (size_t)c.nu * c.nv * V));
    hipError_t e;
    {
        ProfScope prof_("fdk_filter", s);
        k_fdk_filter<<<dim3((unsigned)c.nv, (unsigned)V), 256, 0, s>>>(proj, c, q);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_fdk_views<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(angles, V, views);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t N = grid_size(g);
    {
        ProfScope prof_("fdk_backproject", s);
        k_fdk_bp<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(q, c, V, views, g, vol);
    }
    return hipGetLastError();
}

}  // namespace pmf
