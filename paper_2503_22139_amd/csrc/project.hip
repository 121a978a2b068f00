// project.hip -- cone-beam line integrals (Eq. 6) and their exact adjoint.
//
// Forward: one thread per ray (16x16-pixel tiles per workgroup so that the
// 64 rays of a wave sample neighbouring voxels), midpoint rule in voxel
// units with sample s at u = fma(s, su, bu).
//
// Adjoint: voxel-brick owner, no global atomics.  A workgroup owns a brick of
// the output volume, accumulates in LDS, and visits every ray whose samples
// can touch the brick: the rays through the detector rectangle that bounds
// the brick region's shadow.  A sample contributes to the 8 voxels of its
// cell (i, i+1 per axis), so the brick takes exactly the samples whose cell
// index lies in [B0-1, B0+S-1] on every axis; each ray's sample positions
// come from one per-ray table, so every brick sees bit-identical samples and
// no sample is lost or counted twice.
#include <math.h>

#include "pmf_internal.h"

namespace pmf {

// Per-ray set-up of the midpoint rule, in double precision (a few dozen
// operations per ray against hundreds of samples).  Kept free of FMA
// contraction so every kernel that calls it gets identical bits.
__device__ __attribute__((noinline)) RayK ray_setup(const GridK &g, const ConeK &c, double ct,
                                                     double st, int iu, int iv) {
#pragma clang fp contract(off)
    const double o0 = c.sad * ct, o1 = c.sad * st;
    const double a = ((double)iu - 0.5 * (double)(c.nu - 1) + c.off_u) * c.du;
    const double b = ((double)iv - 0.5 * (double)(c.nv - 1) + c.off_v) * c.dv;
    const double p0 = -(c.sdd - c.sad) * ct + a * (-st);
    const double p1 = -(c.sdd - c.sad) * st + a * ct;
    double d[3] = {p0 - o0, p1 - o1, b};
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] /= len;
    d[1] /= len;
    d[2] /= len;
    const double o[3] = {o0, o1, 0.0};
    double t0 = -INFINITY, t1 = INFINITY;
    bool miss = false;
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < c.lo[k] || o[k] > c.hi[k]) miss = true;
            continue;
        }
        double ta = (c.lo[k] - o[k]) / d[k], tb = (c.hi[k] - o[k]) / d[k];
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
    RayK r;
    if (L > 0.0) {
        double ns = ceil(L / c.step);
        if (ns < 1.0) ns = 1.0;
        r.n = (int)ns;
        const double delta = L / ns;
        r.delta = (float)delta;
        const double tm = t0 + 0.5 * delta;
        for (int k = 0; k < 3; ++k) {
            r.bu[k] = (float)((o[k] + tm * d[k] - g.c0d[k]) / g.hd[k]);
            r.su[k] = (float)(delta * d[k] / g.hd[k]);
        }
    } else {
        r.n = 0;
        r.delta = 0.0f;
        for (int k = 0; k < 3; ++k) {
            r.bu[k] = 0.0f;
            r.su[k] = 0.0f;
        }
    }
    return r;
}

constexpr int PT = 16;  // forward pixel tile edge

__global__ __launch_bounds__(256) void k_project(const float *__restrict__ vol, int64_t stride,
                                                 GridK g, ConeK c,
                                                 const float *__restrict__ angles,
                                                 float *__restrict__ proj, int tiles_u) {
    const int v = blockIdx.y;
    const int tu = blockIdx.x % tiles_u, tv = blockIdx.x / tiles_u;
    const int iu = tu * PT + (threadIdx.x & (PT - 1));
    const int iv = tv * PT + (threadIdx.x / PT);
    if (iu >= c.nu || iv >= c.nv) return;
    const double th = (double)angles[v];
    const RayK r = ray_setup(g, c, cos(th), sin(th), iu, iv);
    const float *__restrict__ vv = vol + (int64_t)v * stride;
    float acc = 0.0f;
    for (int s = 0; s < r.n; ++s) {
        const float sf = (float)s;
        acc += sample_u(vv, g.n, fmaf(sf, r.su[0], r.bu[0]), fmaf(sf, r.su[1], r.bu[1]),
                        fmaf(sf, r.su[2], r.bu[2]));
    }
    proj[((int64_t)v * c.nv + iv) * c.nu + iu] = acc * r.delta;
}

__global__ __launch_bounds__(256) void k_ray_table(GridK g, ConeK c,
                                                   const float *__restrict__ angles, int V,
                                                   RayK *__restrict__ out) {
    const int64_t npix = (int64_t)c.nu * c.nv;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npix * V) return;
    const int v = (int)(q / npix);
    const int p = (int)(q % npix);
    const double th = (double)angles[v];
    out[q] = ray_setup(g, c, cos(th), sin(th), p % c.nu, p / c.nu);
}

// Bounding detector rectangle of the shadow of a world box (double).
__device__ void shadow_rect(const ConeK &c, double ct, double st, const double lo[3],
                            const double hi[3], int &u0, int &u1, int &v0, int &v1) {
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    for (int q = 0; q < 8; ++q) {
        const double x0 = (q & 4) ? hi[0] : lo[0];
        const double x1 = (q & 2) ? hi[1] : lo[1];
        const double x2 = (q & 1) ? hi[2] : lo[2];
        const double depth = x0 * ct + x1 * st;
        const double lat = -x0 * st + x1 * ct;
        const double mag = c.sdd / (c.sad - depth);
        const double fu = lat * mag / c.du + 0.5 * (double)(c.nu - 1) - c.off_u;
        const double fv = x2 * mag / c.dv + 0.5 * (double)(c.nv - 1) - c.off_v;
        umin = fmin(umin, fu);
        umax = fmax(umax, fu);
        vmin = fmin(vmin, fv);
        vmax = fmax(vmax, fv);
    }
    u0 = (int)fmax(floor(umin) - 1.0, 0.0);
    u1 = (int)fmin(ceil(umax) + 1.0, (double)(c.nu - 1));
    v0 = (int)fmax(floor(vmin) - 1.0, 0.0);
    v1 = (int)fmin(ceil(vmax) + 1.0, (double)(c.nv - 1));
}

// g_vol (per view, or summed over views when sum_views) of one brick.
__global__ __launch_bounds__(256) void k_project_bwd(const float *__restrict__ g_proj, GridK g,
                                                     ConeK c, const float *__restrict__ angles,
                                                     const RayK *__restrict__ rays, int V,
                                                     float *__restrict__ g_vol, int64_t stride,
                                                     int S0, int S1, int S2, int nb1, int nb2,
                                                     int sum_views) {
    extern __shared__ float acc[];
    const int nvox = S0 * S1 * S2;
    const int bid = blockIdx.x;
    const int b2 = bid % nb2, b1 = (bid / nb2) % nb1, b0 = bid / (nb2 * nb1);
    const int B[3] = {b0 * S0, b1 * S1, b2 * S2};
    const int S[3] = {S0, S1, S2};
    for (int i = threadIdx.x; i < nvox; i += blockDim.x) acc[i] = 0.0f;

    int clo[3], chi[3];
    float ulo[3], uhi[3];
    double wlo[3], whi[3];
    for (int a = 0; a < 3; ++a) {
        clo[a] = max(B[a] - 1, 0);
        chi[a] = min(B[a] + S[a] - 1, g.n[a] - 2);
        ulo[a] = clo[a] == 0 ? -0.5f : (float)clo[a];
        uhi[a] = chi[a] == g.n[a] - 2 ? (float)g.n[a] - 0.5f : (float)(chi[a] + 1);
        wlo[a] = g.c0d[a] + ((double)ulo[a] - 0.5) * g.hd[a];
        whi[a] = g.c0d[a] + ((double)uhi[a] + 0.5) * g.hd[a];
    }
    __syncthreads();

    const int vb = sum_views ? 0 : blockIdx.y;
    const int ve = sum_views ? V : blockIdx.y + 1;
    for (int v = vb; v < ve; ++v) {
        const double th = (double)angles[v];
        const double ct = cos(th), st = sin(th);
        int u0, u1, v0, v1;
        shadow_rect(c, ct, st, wlo, whi, u0, u1, v0, v1);
        if (u1 < u0 || v1 < v0) continue;
        const int rw = u1 - u0 + 1;
        const int nr = rw * (v1 - v0 + 1);
        for (int q = threadIdx.x; q < nr; q += blockDim.x) {
            const int iu = u0 + q % rw, iv = v0 + q / rw;
            const int64_t pix = ((int64_t)v * c.nv + iv) * c.nu + iu;
            const RayK r = rays[pix];
            if (r.n == 0) continue;
            const float gp = g_proj[pix] * r.delta;
            if (gp == 0.0f) continue;
            float smin = 0.0f, smax = (float)(r.n - 1);
            bool skip = false;
            for (int a = 0; a < 3; ++a) {
                if (r.su[a] != 0.0f) {
                    const float ta = (ulo[a] - r.bu[a]) / r.su[a];
                    const float tb = (uhi[a] - r.bu[a]) / r.su[a];
                    smin = fmaxf(smin, fminf(ta, tb));
                    smax = fminf(smax, fmaxf(ta, tb));
                } else if (r.bu[a] < ulo[a] - 1.0f || r.bu[a] > uhi[a] + 1.0f) {
                    skip = true;
                }
            }
            if (skip || smin > smax + 2.0f) continue;
            const int s0 = max(0, (int)floorf(smin) - 1);
            const int s1 = min(r.n - 1, (int)ceilf(smax) + 1);
            for (int s = s0; s <= s1; ++s) {
                const float sf = (float)s;
                int i0, i1, i2;
                float f0, f1, f2;
                if (!axis_cell(fmaf(sf, r.su[0], r.bu[0]), g.n[0], i0, f0) ||
                    !axis_cell(fmaf(sf, r.su[1], r.bu[1]), g.n[1], i1, f1) ||
                    !axis_cell(fmaf(sf, r.su[2], r.bu[2]), g.n[2], i2, f2))
                    continue;
                if (i0 < clo[0] || i0 > chi[0] || i1 < clo[1] || i1 > chi[1] || i2 < clo[2] ||
                    i2 > chi[2])
                    continue;
                const float w0[2] = {1.0f - f0, f0}, w1[2] = {1.0f - f1, f1},
                            w2[2] = {1.0f - f2, f2};
                const int l0 = i0 - B[0], l1 = i1 - B[1], l2 = i2 - B[2];
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const int x = l0 + dx;
                    if (x < 0 || x >= S0) continue;
#pragma unroll
                    for (int dy = 0; dy < 2; ++dy) {
                        const int y = l1 + dy;
                        if (y < 0 || y >= S1) continue;
                        const float wxy = gp * w0[dx] * w1[dy];
#pragma unroll
                        for (int dz = 0; dz < 2; ++dz) {
                            const int z = l2 + dz;
                            if (z < 0 || z >= S2) continue;
                            atomicAdd(&acc[(x * S1 + y) * S2 + z], wxy * w2[dz]);
                        }
                    }
                }
            }
        }
        if (!sum_views) break;
    }
    __syncthreads();
    float *out = g_vol + (sum_views ? 0 : (int64_t)blockIdx.y * stride);
    for (int i = threadIdx.x; i < nvox; i += blockDim.x) {
        const int z = i % S2, y = (i / S2) % S1, x = i / (S2 * S1);
        const int gx = B[0] + x, gy = B[1] + y, gz = B[2] + z;
        if (gx < g.n[0] && gy < g.n[1] && gz < g.n[2])
            out[((int64_t)gx * g.n[1] + gy) * g.n[2] + gz] = acc[i];
    }
}

hipError_t launch_project(const float *vol, int64_t stride, const GridK &g, const ConeK &c,
                          const float *angles, int V, float *proj, hipStream_t s) {
    const int tu = (c.nu + PT - 1) / PT, tv = (c.nv + PT - 1) / PT;
    dim3 grid((unsigned)(tu * tv), (unsigned)V);
    {
        ProfScope prof_("project", s);
        k_project<<<grid, 256, 0, s>>>(vol, stride, g, c, angles, proj, tu);
    }
    return hipGetLastError();
}

static const int BWD_S[3] = {16, 16, 16};

size_t project_bwd_workspace(const pmf_cone_t &c, int V) {
    return align256(sizeof(RayK) * (size_t)c.nu * (size_t)c.nv * (size_t)V);
}

hipError_t launch_project_bwd(const float *g_proj, const GridK &g, const ConeK &c,
                              const float *angles, int V, float *g_vol, int64_t stride, void *ws,
                              hipStream_t s) {
    RayK *rays = (RayK *)ws;
    const int64_t nr = (int64_t)c.nu * c.nv * V;
    {
        ProfScope prof_("ray_table", s);
        k_ray_table<<<(unsigned)((nr + 255) / 256), 256, 0, s>>>(g, c, angles, V, rays);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int S[3];
    int nb[3];
    for (int a = 0; a < 3; ++a) {
        S[a] = BWD_S[a] < g.n[a] ? BWD_S[a] : g.n[a];
        nb[a] = (g.n[a] + S[a] - 1) / S[a];
    }
    const int sum_views = stride == 0;
    dim3 grid((unsigned)(nb[0] * nb[1] * nb[2]), sum_views ? 1u : (unsigned)V);
    const size_t lds = sizeof(float) * (size_t)S[0] * S[1] * S[2];
    {
        ProfScope prof_("project_bwd", s);
        k_project_bwd<<<grid, 256, lds, s>>>(g_proj, g, c, angles, rays, V, g_vol, stride, S[0], S[1],
                                             S[2], nb[1], nb[2], sum_views);
    }
    return hipGetLastError();
}

}  // namespace pmf
