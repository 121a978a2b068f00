// loss.hip -- L2 projection loss of a batch of views and its gradient.
#include "pmf_internal.h"

namespace pmf {

constexpr int L2_BLOCKS = 512;

__global__ __launch_bounds__(256) void k_l2(const float *__restrict__ p,
                                            const float *__restrict__ t, int64_t n, float gscale,
                                            float *__restrict__ g, float *__restrict__ partial) {
    float acc = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float r = p[i] - t[i];
        acc = fmaf(r, r, acc);
        if (g) g[i] = gscale * r;
    }
    __shared__ float red[4];
    acc = wave_sum_lane63(acc);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_l2_final(const float *__restrict__ partial, int nb, float inv_v,
                           float *__restrict__ loss) {
    if (threadIdx.x != 0) return;
    float s = 0.0f;
    for (int i = 0; i < nb; ++i) s += partial[i];
    *loss = s * inv_v;
}

size_t l2_workspace(int64_t npix, int V) {
    (void)npix;
    (void)V;
    return align256(sizeof(float) * L2_BLOCKS);
}

hipError_t launch_l2(const float *proj, const float *target, int64_t npix, int V, float *loss,
                     float *g, void *ws, hipStream_t s) {
    const int64_t n = npix * V;
    int nb = (int)((n + 255) / 256);
    if (nb > L2_BLOCKS) nb = L2_BLOCKS;
    if (nb < 1) nb = 1;
    float *partial = (float *)ws;
    {
        ProfScope prof_("l2_loss", s);
        k_l2<<<(unsigned)nb, 256, 0, s>>>(proj, target, n, 2.0f / (float)V, g, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        ProfScope prof_("l2_loss_final", s);
        k_l2_final<<<1, 64, 0, s>>>(partial, nb, 1.0f / (float)V, loss);
    }
    return hipGetLastError();
}

}  // namespace pmf
