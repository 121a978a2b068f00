// warp.hip -- the motion-compensated warp of Eq. 2 and its adjoint.
//
// One thread per voxel of the output grid; the sample point x_j + d is taken
// in voxel units as i_a + t_a, t_a = d_a / h_a, its cell decided from t_a
// (disp_cell).  The adjoint writes g_dvf directly (one owner per entry) and
// scatters g_ref onto the 8 corners of each sample in 64-bit fixed point
// (fix_add, scale from the largest |g_out|), so g_ref does not depend on the
// order of the additions; a last pass converts it to float.
#include "pmf_internal.h"

namespace pmf {

__global__ __launch_bounds__(256) void k_warp(const float *__restrict__ ref, GridK g,
                                              const float *__restrict__ dvf, int V,
                                              float *__restrict__ out) {
    const int64_t N = grid_size(g);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int iz = (int)(j % g.n[2]);
    const int iy = (int)((j / g.n[2]) % g.n[1]);
    const int ix = (int)(j / ((int64_t)g.n[2] * g.n[1]));
    for (int v = 0; v < V; ++v) {
        const float *d = dvf + (int64_t)v * 3 * N;
        const float t0 = d[j] * g.inv_h[0], t1 = d[N + j] * g.inv_h[1],
                    t2 = d[2 * N + j] * g.inv_h[2];
        out[(int64_t)v * N + j] = sample_disp(ref, g.n, ix, iy, iz, t0, t1, t2);
    }
}

__global__ __launch_bounds__(256) void k_warp_bwd(const float *__restrict__ ref, GridK g,
                                                  const float *__restrict__ dvf, int V,
                                                  const float *__restrict__ g_out,
                                                  const uint32_t *__restrict__ gmax,
                                                  long long *__restrict__ fix,
                                                  float *__restrict__ g_dvf) {
    const int64_t N = grid_size(g);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int iz = (int)(j % g.n[2]);
    const int iy = (int)((j / g.n[2]) % g.n[1]);
    const int ix = (int)(j / ((int64_t)g.n[2] * g.n[1]));
    const int s1 = g.n[2], s0 = g.n[1] * g.n[2];
    const double fscale = fix_scale(*gmax);
    for (int v = 0; v < V; ++v) {
        const float *d = dvf + (int64_t)v * 3 * N;
        const float t0 = d[j] * g.inv_h[0], t1 = d[N + j] * g.inv_h[1],
                    t2 = d[2 * N + j] * g.inv_h[2];
        const float go = g_out[(int64_t)v * N + j];
        float *gd = g_dvf + (int64_t)v * 3 * N;
        int i0, i1, i2;
        float f0, f1, f2;
        if (!disp_cell(ix, t0, g.n[0], i0, f0) || !disp_cell(iy, t1, g.n[1], i1, f1) ||
            !disp_cell(iz, t2, g.n[2], i2, f2)) {
            gd[j] = 0.0f;
            gd[N + j] = 0.0f;
            gd[2 * N + j] = 0.0f;
            continue;
        }
        const int64_t base = ((int64_t)i0 * g.n[1] + i1) * g.n[2] + i2;
        const float *p = ref + base;
        const float c000 = p[0], c001 = p[1], c010 = p[s1], c011 = p[s1 + 1];
        const float c100 = p[s0], c101 = p[s0 + 1], c110 = p[s0 + s1], c111 = p[s0 + s1 + 1];
        // derivative of the trilinear blend along each axis (per voxel unit)
        const float a00 = lerp1(c000, c001, f2), a01 = lerp1(c010, c011, f2);
        const float a10 = lerp1(c100, c101, f2), a11 = lerp1(c110, c111, f2);
        const float dx = lerp1(a10, a11, f1) - lerp1(a00, a01, f1);
        const float dy = lerp1(a01, a11, f0) - lerp1(a00, a10, f0);
        const float b00 = lerp1(c000, c010, f1), b01 = lerp1(c001, c011, f1);
        const float b10 = lerp1(c100, c110, f1), b11 = lerp1(c101, c111, f1);
        const float dz = lerp1(b01, b11, f0) - lerp1(b00, b10, f0);
        gd[j] = go * dx * g.inv_h[0] * disp_free(ix, t0, g.n[0]);
        gd[N + j] = go * dy * g.inv_h[1] * disp_free(iy, t1, g.n[1]);
        gd[2 * N + j] = go * dz * g.inv_h[2] * disp_free(iz, t2, g.n[2]);
        if (go == 0.0f) continue;
        const float w0[2] = {1.0f - f0, f0}, w1[2] = {1.0f - f1, f1}, w2[2] = {1.0f - f2, f2};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    fix_add(&fix[base + a * s0 + b * s1 + c], (double)(go * w0[a] * w1[b] * w2[c]),
                            fscale);
    }
}

hipError_t launch_warp(const float *ref, const GridK &g, const float *dvf, int V, float *out,
                       hipStream_t s) {
    const int64_t N = grid_size(g);
    {
        ProfScope prof_("warp", s);
        k_warp<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(ref, g, dvf, V, out);
    }
    return hipGetLastError();
}

// Workspace: the 64-bit fixed-point g_ref, then the largest |g_out|.
size_t warp_bwd_workspace(const GridK &g) {
    return align256(sizeof(long long) * (size_t)grid_size(g)) + align256(sizeof(uint32_t));
}

hipError_t launch_warp_bwd(const float *ref, const GridK &g, const float *dvf, int V,
                           const float *g_out, float *g_ref, float *g_dvf, void *ws,
                           hipStream_t s) {
    const int64_t N = grid_size(g);
    long long *fix = (long long *)ws;
    uint32_t *gmax = (uint32_t *)((char *)ws + align256(sizeof(long long) * (size_t)N));
    hipError_t e = launch_fill_i32((int32_t *)fix, 2 * N, 0, s);
    if (e != hipSuccess) return e;
    if ((e = launch_absmax(g_out, N * V, gmax, s)) != hipSuccess) return e;
    {
        ProfScope prof_("warp_bwd", s);
        k_warp_bwd<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(ref, g, dvf, V, g_out, gmax, fix,
                                                                g_dvf);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_fix_to_float(fix, N, gmax, false, g_ref, s);
}

}  // namespace pmf
