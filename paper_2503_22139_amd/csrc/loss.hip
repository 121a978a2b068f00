// loss.hip -- L2 projection loss of a batch of views and its gradient.
#include "pmf_internal.h"

namespace pmf {

constexpr int L2_BLOCKS = 2048;

// Per-block partial sums of squared residuals, and the residual gradient.
// VEC: the three arrays are 16-byte aligned and the bulk moves as float4
// (the last n % 4 elements go through the scalar loop).
template <bool VEC>
__global__ __launch_bounds__(256) void k_l2(const float *__restrict__ p,
                                            const float *__restrict__ t, int64_t n, float gscale,
                                            float *__restrict__ g, float *__restrict__ partial) {
    float acc = 0.0f;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i0 = tid;
    if (VEC) {
        const int64_t n4 = n >> 2;
        for (int64_t i = tid; i < n4; i += stride) {
            const float4 a = ((const float4 *)p)[i], b = ((const float4 *)t)[i];
            const float4 r = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
            acc = fmaf(r.x, r.x, acc);
            acc = fmaf(r.y, r.y, acc);
            acc = fmaf(r.z, r.z, acc);
            acc = fmaf(r.w, r.w, acc);
            if (g)
                ((float4 *)g)[i] =
                    make_float4(gscale * r.x, gscale * r.y, gscale * r.z, gscale * r.w);
        }
        i0 = 4 * n4 + tid;
    }
    for (int64_t i = i0; i < n; i += stride) {
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

// One wave: the partials in a fixed order, scaled.
__global__ __launch_bounds__(64) void k_l2_final(const float *__restrict__ partial, int nb,
                                                 float inv_v, float *__restrict__ loss) {
    const float s = wave_sum_partials(partial, nb);
    if (threadIdx.x == 63) *loss = s * inv_v;
}

size_t l2_workspace(int64_t npix, int V) {
    (void)npix;
    (void)V;
    return align256(sizeof(float) * L2_BLOCKS);
}

hipError_t launch_l2(const float *proj, const float *target, int64_t npix, int V, float *loss,
                     float *g, void *ws, hipStream_t s) {
    const int64_t n = npix * V;
    const bool vec =
        (((uintptr_t)proj | (uintptr_t)target | (uintptr_t)g) & 15) == 0 && n >= 4;
    const int64_t items = vec ? n / 4 : n;
    int nb = (int)std::min<int64_t>((items + 255) / 256, L2_BLOCKS);
    if (nb < 1) nb = 1;
    float *partial = (float *)ws;
    {
        ProfScope prof_("l2_loss", s);
        if (vec)
            k_l2<true><<<(unsigned)nb, 256, 0, s>>>(proj, target, n, 2.0f / (float)V, g, partial);
        else
            k_l2<false><<<(unsigned)nb, 256, 0, s>>>(proj, target, n, 2.0f / (float)V, g, partial);
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
