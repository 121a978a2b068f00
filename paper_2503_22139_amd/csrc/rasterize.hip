// rasterize.hip -- the X-ray Gaussian rasterizer of Stage 1 (Sec. 2.2,
// Eq. 7-9) and its adjoint.
//
// Per view, each 3-D Gaussian (mean p, Sigma = R(q) diag(s^2) R(q)^T, density
// rho) is mapped to a 2-D Gaussian on the detector by the local affine
// approximation of the projective map phi (Eq. 8): t = W (p - o) in the
// source-centred frame (u, v, central ray), phi(t) = (SDD t_u / (t_d du) +
// cu, SDD t_v / (t_d dv) + cv, |t|), J = d phi / d t at t, Sigma~ = J W Sigma
// W^T J^T; integrating along the ray coordinate (Eq. 9) leaves centre
// phi_01(t), covariance Sigma^ (top-left 2 x 2 of Sigma~) and amplitude
// rho sqrt(2 pi |Sigma~| / |Sigma^|).  A pixel's value is the sum of the
// 2-D Gaussians at its centre, each truncated to (x - mu)^T Sigma^-1 (x - mu)
// <= k^2 (k = inf: untruncated); Gaussians not in front of the source are
// skipped.  Geometry and pixel centres are those of the ray-march projector.
//
// Forward: per-(view, Gaussian) set-up in double, tile binning (16 x 16-pixel
// tiles; a Gaussian whose truncation box covers more than RS_TMAX tiles goes
// to a list of large splats), then one workgroup per tile: Gaussians staged
// in LDS, one pixel per thread, summed in fixed point (bit-reproducible),
// the large splats that reach the tile after its list.  Adjoint: the same
// binning; per tile each wave reduces its pixels' contributions to the six
// 2-D parameters (amplitude, centre, conic) of a Gaussian, and the tile
// writes the sum of its waves (fixed order) to a partial per list entry; a
// gather pass then sums each Gaussian's partials in tile order (no atomics),
// and per (view, Gaussian) the chain rule goes back to (p, s, q, rho) in
// double, summed over views in order.
#include <math.h>

#include "pmf_internal.h"

namespace pmf {

constexpr int RS_T = 16;                // tile edge (pixels)
constexpr int RS_THREADS = RS_T * RS_T;
constexpr int RS_TMAX = 16;             // tiles per Gaussian on the tile path
// Tile counters one per 128-byte line: the count's device-scope atomics
// contend per line.
constexpr int RS_CSTRIDE = 32;

// 2-D splat of one (view, Gaussian): centre, conic (Sigma^-1 = [[a, b], [b, c]]),
// amplitude, and its tile rectangle (empty when lo > hi).
struct alignas(16) SplatP {
    float mu_u, mu_v, a, b;
    float c, rho;
    int16_t tu0, tv0, tu1, tv1;
};

struct RastGeo {
    double sad, sdd, du, dv, off_u, off_v;
    int nu, nv, tiles_u, tiles_v;
    float k;        // truncation radius (inf: none)
};

// Per (view, Gaussian) quantities in double: the view frame, J, Sigma~.
struct SplatD {
    bool ok;
    double t[3], nt, W[3][3], J[3][3], M[3][3], R[3][3], Sig[3][3], St[3][3];
    double mu[2], Sh[3];       // Sigma^ (s00, s01, s11)
    double det2, det3, amp;    // amp = sqrt(2 pi det3 / det2)
    double qh[4], qn;
};

__device__ void splat_setup(const RastGeo &G, double th, const float *p, const float *s,
                            const float *q, SplatD &D) {
    const double ct = cos(th), st = sin(th);
    const double o[3] = {G.sad * ct, G.sad * st, 0.0};
    const double W[3][3] = {{-st, ct, 0.0}, {0.0, 0.0, 1.0}, {-ct, -st, 0.0}};
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = (double)p[a] - o[a];
    for (int r = 0; r < 3; ++r) {
        D.t[r] = W[r][0] * x[0] + W[r][1] * x[1] + W[r][2] * x[2];
        for (int c = 0; c < 3; ++c) D.W[r][c] = W[r][c];
    }
    D.ok = D.t[2] > 0.0;
    const double td = D.ok ? D.t[2] : 1.0;
    const double su = G.sdd / G.du, sv = G.sdd / G.dv;
    D.nt = sqrt(D.t[0] * D.t[0] + D.t[1] * D.t[1] + D.t[2] * D.t[2]);
    D.mu[0] = su * D.t[0] / td + 0.5 * (G.nu - 1) - G.off_u;
    D.mu[1] = sv * D.t[1] / td + 0.5 * (G.nv - 1) - G.off_v;
    double J[3][3] = {{su / td, 0.0, -su * D.t[0] / (td * td)},
                      {0.0, sv / td, -sv * D.t[1] / (td * td)},
                      {D.t[0] / D.nt, D.t[1] / D.nt, D.t[2] / D.nt}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            D.J[r][c] = J[r][c];
            D.M[r][c] = J[r][0] * W[0][c] + J[r][1] * W[1][c] + J[r][2] * W[2][c];
        }
    // Sigma = R diag(s^2) R^T, normalised quaternion (w, x, y, z)
    D.qn = sqrt((double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3]);
    for (int k = 0; k < 4; ++k) D.qh[k] = q[k] / D.qn;
    const double w = D.qh[0], xq = D.qh[1], y = D.qh[2], z = D.qh[3];
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (xq * y - w * z), 2 * (xq * z + w * y)},
                            {2 * (xq * y + w * z), 1 - 2 * (xq * xq + z * z), 2 * (y * z - w * xq)},
                            {2 * (xq * z - w * y), 2 * (y * z + w * xq), 1 - 2 * (xq * xq + y * y)}};
    const double s2[3] = {(double)s[0] * s[0], (double)s[1] * s[1], (double)s[2] * s[2]};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            D.R[r][c] = R[r][c];
            D.Sig[r][c] = R[r][0] * s2[0] * R[c][0] + R[r][1] * s2[1] * R[c][1] + R[r][2] * s2[2] * R[c][2];
        }
    double MS[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            MS[r][c] = D.M[r][0] * D.Sig[0][c] + D.M[r][1] * D.Sig[1][c] + D.M[r][2] * D.Sig[2][c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            D.St[r][c] = MS[r][0] * D.M[c][0] + MS[r][1] * D.M[c][1] + MS[r][2] * D.M[c][2];
    D.Sh[0] = D.St[0][0];
    D.Sh[1] = D.St[0][1];
    D.Sh[2] = D.St[1][1];
    D.det2 = D.Sh[0] * D.Sh[2] - D.Sh[1] * D.Sh[1];
    D.det3 = D.St[0][0] * (D.St[1][1] * D.St[2][2] - D.St[1][2] * D.St[2][1]) -
             D.St[0][1] * (D.St[1][0] * D.St[2][2] - D.St[1][2] * D.St[2][0]) +
             D.St[0][2] * (D.St[1][0] * D.St[2][1] - D.St[1][1] * D.St[2][0]);
    D.ok = D.ok && D.det2 > 0.0 && D.det3 > 0.0;
    D.amp = D.ok ? sqrt(2.0 * M_PI * D.det3 / D.det2) : 0.0;
}

// ------------------------------------------------------------------ binning
// Per (view, Gaussian): the splat and its tile rectangle; counts tiles of
// small rectangles (each count's old value, the pair's place in the tile's
// list, goes to gslot for the fill), lists large ones.
__global__ __launch_bounds__(256) void k_splat_prep(const float *__restrict__ mean,
                                                    const float *__restrict__ scale,
                                                    const float *__restrict__ quat,
                                                    const float *__restrict__ value, int64_t m,
                                                    int V, RastGeo G,
                                                    const float *__restrict__ angles,
                                                    SplatP *__restrict__ sp,
                                                    int *__restrict__ counts,
                                                    int *__restrict__ gslot,
                                                    int *__restrict__ large, int *__restrict__ nlarge) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * V) return;
    const int v = (int)(i / m);
    const int64_t g = i - (int64_t)v * m;
    SplatD D;
    splat_setup(G, (double)angles[v], mean + 3 * g, scale + 3 * g, quat + 4 * g, D);
    SplatP P;
    P.tu0 = P.tv0 = 1;
    P.tu1 = P.tv1 = 0;
    if (D.ok) {
        P.mu_u = (float)D.mu[0];
        P.mu_v = (float)D.mu[1];
        P.a = (float)(D.Sh[2] / D.det2);
        P.b = (float)(-D.Sh[1] / D.det2);
        P.c = (float)(D.Sh[0] / D.det2);
        P.rho = (float)((double)value[g] * D.amp);
        double u0 = 0.0, u1 = G.nu - 1, v0 = 0.0, v1 = G.nv - 1;
        if (isfinite(G.k)) {
            const double ru = G.k * sqrt(D.Sh[0]), rv = G.k * sqrt(D.Sh[2]);
            u0 = fmax(u0, ceil(D.mu[0] - ru));
            u1 = fmin(u1, floor(D.mu[0] + ru));
            v0 = fmax(v0, ceil(D.mu[1] - rv));
            v1 = fmin(v1, floor(D.mu[1] + rv));
        }
        if (u0 <= u1 && v0 <= v1) {
            P.tu0 = (int16_t)((int)u0 / RS_T);
            P.tu1 = (int16_t)((int)u1 / RS_T);
            P.tv0 = (int16_t)((int)v0 / RS_T);
            P.tv1 = (int16_t)((int)v1 / RS_T);
        }
    } else {
        P.mu_u = P.mu_v = P.a = P.b = P.c = P.rho = 0.0f;
    }
    sp[i] = P;
    if (P.tu0 > P.tu1 || P.tv0 > P.tv1) return;
    const int area = (P.tu1 - P.tu0 + 1) * (P.tv1 - P.tv0 + 1);
    if (area > RS_TMAX) {
        large[atomicAdd(nlarge, 1)] = (int)i;
        return;
    }
    int *cv = counts + (int64_t)v * G.tiles_u * G.tiles_v * RS_CSTRIDE;
    int k = 0;
    for (int ty = P.tv0; ty <= P.tv1; ++ty)
        for (int tx = P.tu0; tx <= P.tu1; ++tx)
            gslot[i * RS_TMAX + k++] = atomicAdd(&cv[(ty * G.tiles_u + tx) * RS_CSTRIDE], 1);
}

// Exclusive prefix sum of n counts (RS_CSTRIDE apart; one workgroup, chunks
// of 1024) into dense offsets.
__global__ __launch_bounds__(1024) void k_rast_scan(const int *__restrict__ counts, int64_t n,
                                                    int *__restrict__ offsets) {
    __shared__ int buf[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < n; b += 1024) {
        const int64_t i = b + threadIdx.x;
        const int x = i < n ? counts[i * RS_CSTRIDE] : 0;
        buf[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int y = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < n) offsets[i] = carry + buf[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[n] = carry;
}

// Each (view, Gaussian) writes itself at the places the count drew (no
// atomics) and turns its gslot entries into list positions, in (row,
// column) order, so that the adjoint can sum a Gaussian's per-tile partials
// in a fixed order.
__global__ __launch_bounds__(256) void k_splat_fill(const SplatP *__restrict__ sp, int64_t m,
                                                    int V, RastGeo G,
                                                    const int *__restrict__ offsets,
                                                    int *__restrict__ list,
                                                    int *__restrict__ gslot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * V) return;
    const SplatP P = sp[i];
    if (P.tu0 > P.tu1 || P.tv0 > P.tv1) return;
    if ((P.tu1 - P.tu0 + 1) * (P.tv1 - P.tv0 + 1) > RS_TMAX) return;
    const int v = (int)(i / m);
    const int64_t T = (int64_t)G.tiles_u * G.tiles_v;
    int k = 0;
    for (int ty = P.tv0; ty <= P.tv1; ++ty)
        for (int tx = P.tu0; tx <= P.tu1; ++tx) {
            const int64_t tix = (int64_t)v * T + ty * G.tiles_u + tx;
            const int slot = offsets[tix] + gslot[i * RS_TMAX + k];
            list[slot] = (int)i;
            gslot[i * RS_TMAX + k++] = slot;
        }
}

// Contribution of splat P at pixel (x, y): rho exp(-m/2) inside the ellipse.
__device__ __forceinline__ float splat_at(const SplatP &P, float x, float y, float k2, float &du,
                                          float &dv, float &e) {
    du = x - P.mu_u;
    dv = y - P.mu_v;
    const float m = fmaf(P.a * du, du, fmaf(2.0f * P.b * du, dv, P.c * dv * dv));
    e = m <= k2 ? __expf(-0.5f * m) : 0.0f;
    return P.rho * e;
}

// ------------------------------------------------------------------ forward
// One workgroup per (view, tile), one pixel per thread.  Each pixel sums its
// splats in 32-bit fixed point with the tile's scale 2^30 / S, S = (number of
// splats reaching the tile: its list and the view's large Gaussians) x (their
// largest |amplitude|), so every pixel's sum stays below 2^30: neither the
// integer sums nor S depend on the order in which the binning's atomics
// filled the list, so the images repeat bit for bit.  The large Gaussians (no tile entries) are walked by
// every tile they reach, after its list.
__global__ __launch_bounds__(RS_THREADS) void k_splat_fwd(const SplatP *__restrict__ sp, int64_t m,
                                                         RastGeo G,
                                                         const int *__restrict__ offsets,
                                                         const int *__restrict__ list,
                                                         const int *__restrict__ large,
                                                         const int *__restrict__ nlarge,
                                                         float *__restrict__ proj) {
    __shared__ SplatP sh[RS_THREADS];
    __shared__ float red[RS_THREADS / 64];
    __shared__ int cnt[RS_THREADS / 64];
    const int64_t T = (int64_t)G.tiles_u * G.tiles_v;
    const int64_t tix = blockIdx.x;
    const int v = (int)(tix / T), t = (int)(tix - (int64_t)v * T);
    const int tx = t % G.tiles_u, ty = t / G.tiles_u;
    const int x = tx * RS_T + (threadIdx.x % RS_T);
    const int y = ty * RS_T + (threadIdx.x / RS_T);
    const float k2 = G.k * G.k;
    const int b = offsets[tix], e = offsets[tix + 1];
    const int nl = *nlarge;
    auto reaches = [&](const SplatP &P) {
        return P.tu0 <= tx && tx <= P.tu1 && P.tv0 <= ty && ty <= P.tv1;
    };
    // S = (splats reaching the tile) x (their largest |amplitude|): an
    // order-independent bound of every pixel's sum
    float mx = 0.0f;
    int nh = 0;
    for (int q = b + (int)threadIdx.x; q < e; q += RS_THREADS) mx = fmaxf(mx, fabsf(sp[list[q]].rho));
    for (int q = (int)threadIdx.x; q < nl; q += RS_THREADS) {
        const int64_t i = large[q];
        if (i / m == v && reaches(sp[i])) {
            mx = fmaxf(mx, fabsf(sp[i].rho));
            ++nh;
        }
    }
    mx = wave_max(mx);
    for (int o = 32; o > 0; o >>= 1) nh += __shfl_xor(nh, o, 64);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = mx;
        cnt[threadIdx.x >> 6] = nh;
    }
    __syncthreads();
    const float S = (float)((e - b) + cnt[0] + cnt[1] + cnt[2] + cnt[3]) *
                    fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    const float scale = S > 0.0f ? 1073741824.0f / (S * 1.0001f) : 0.0f;
    int acc = 0;
    for (int c0 = b; c0 < e; c0 += RS_THREADS) {
        const int n = min(RS_THREADS, e - c0);
        if ((int)threadIdx.x < n) sh[threadIdx.x] = sp[list[c0 + threadIdx.x]];
        __syncthreads();
        for (int j = 0; j < n; ++j) {
            float du, dv, ex;
            acc += __float2int_rn(splat_at(sh[j], (float)x, (float)y, k2, du, dv, ex) * scale);
        }
        __syncthreads();
    }
    for (int q = 0; q < nl; ++q) {
        const int64_t i = large[q];
        if (i / m != v) continue;
        const SplatP P = sp[i];
        if (!reaches(P)) continue;
        float du, dv, ex;
        acc += __float2int_rn(splat_at(P, (float)x, (float)y, k2, du, dv, ex) * scale);
    }
    if (x < G.nu && y < G.nv)
        proj[((int64_t)v * G.nv + y) * G.nu + x] = scale > 0.0f ? (float)acc / scale : 0.0f;
}

// ------------------------------------------------------------------ adjoint
// d L / d(rho^, mu_u, mu_v, a, b, c) of a splat from pixel (x, y) with dL/dI = g.
__device__ __forceinline__ void splat_grad(const SplatP &P, float x, float y, float k2, float g,
                                           float out[6]) {
    float du, dv, e;
    splat_at(P, x, y, k2, du, dv, e);
    const float ge = g * e, gre = ge * P.rho;
    out[0] = ge;
    out[1] = gre * fmaf(P.a, du, P.b * dv);
    out[2] = gre * fmaf(P.b, du, P.c * dv);
    out[3] = -0.5f * gre * du * du;
    out[4] = -gre * du * dv;
    out[5] = -0.5f * gre * dv * dv;
}

// Per tile: each wave reduces its 64 pixels' six splat gradients per
// Gaussian into its LDS slot (zeros when no pixel of the wave is inside any
// of the five ellipses reduced together); the four slots are added in a
// fixed order and written to part[list entry] -- no atomics.
constexpr int RB_CHUNK = 64;      // Gaussians per LDS chunk in the adjoint
constexpr int RB_SPLIT = 8;       // workgroups sharing one tile's list in the adjoint

__global__ __launch_bounds__(RS_THREADS) void k_splat_bwd(const SplatP *__restrict__ sp, RastGeo G,
                                                         const int *__restrict__ offsets,
                                                         const int *__restrict__ list,
                                                         const float *__restrict__ g_proj,
                                                         float *__restrict__ part) {
    __shared__ SplatP sh[RB_CHUNK];
    __shared__ float red[RS_THREADS / 64][RB_CHUNK][6];
    const int wave = threadIdx.x >> 6;
    const int64_t T = (int64_t)G.tiles_u * G.tiles_v;
    const int64_t tix = blockIdx.x;
    const int v = (int)(tix / T), t = (int)(tix - (int64_t)v * T);
    const int x = (t % G.tiles_u) * RS_T + (threadIdx.x % RS_T);
    const int y = (t / G.tiles_u) * RS_T + (threadIdx.x / RS_T);
    const bool in = x < G.nu && y < G.nv;
    const float gp = in ? g_proj[((int64_t)v * G.nv + y) * G.nu + x] : 0.0f;
    const float k2 = G.k * G.k;
    const int lane = threadIdx.x & 63;
    const int b = offsets[tix], e = offsets[tix + 1];
    // the tile's list is dealt over gridDim.y workgroups chunk by chunk (each
    // entry has its own partial, so they need no reduction)
    for (int c0 = b + (int)blockIdx.y * RB_CHUNK; c0 < e; c0 += (int)gridDim.y * RB_CHUNK) {
        const int n = min(RB_CHUNK, e - c0);
        if ((int)threadIdx.x < n) sh[threadIdx.x] = sp[list[c0 + threadIdx.x]];
        __syncthreads();
        // five Gaussians at a time: their 30 wave sums come from one 32-value
        // reduce-scatter (~33 additions instead of 30 six-step reductions)
        for (int j0 = 0; j0 < n; j0 += 5) {
            float xv[32];
            bool any = false;
#pragma unroll
            for (int jj = 0; jj < 5; ++jj) {
                float o[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (j0 + jj < n) splat_grad(sh[j0 + jj], (float)x, (float)y, k2, gp, o);
                any = any || o[0] != 0.0f;
#pragma unroll
                for (int q = 0; q < 6; ++q) xv[q * 5 + jj] = o[q];
            }
            xv[30] = 0.0f;
            xv[31] = 0.0f;
            const int idx = scatter32_index(lane);
            float r = 0.0f;
            if (__ballot(any) != 0) r = wave_reduce_scatter32(xv, lane);   // wave-uniform
            const int jj = idx % 5, q = idx / 5;
            if (lane < 32 && idx < 30 && j0 + jj < n) red[wave][j0 + jj][q] = r;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n * 6; i += RS_THREADS) {
            const int j = i / 6, q = i - 6 * j;
            part[(int64_t)c0 * 6 + i] = (red[0][j][q] + red[1][j][q]) + (red[2][j][q] + red[3][j][q]);
        }
        __syncthreads();
    }
}

// acc6 of every tile-path (view, Gaussian): the sum of its per-tile partials
// in tile order (0 for splats that reach no pixel); large-list splats are
// left to k_splat_large_bwd.
__global__ __launch_bounds__(256) void k_splat_gather(const SplatP *__restrict__ sp, int64_t mv,
                                                      const int *__restrict__ gslot,
                                                      const float *__restrict__ part,
                                                      float *__restrict__ acc6) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mv) return;
    const SplatP P = sp[i];
    int area = 0;
    if (P.tu0 <= P.tu1 && P.tv0 <= P.tv1) area = (P.tu1 - P.tu0 + 1) * (P.tv1 - P.tv0 + 1);
    if (area > RS_TMAX) return;
    float o[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int k = 0; k < area; ++k) {
        const float *pk = part + (int64_t)gslot[i * RS_TMAX + k] * 6;
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] += pk[q];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) acc6[i * 6 + q] = o[q];
}

// Large-list Gaussians: one workgroup sums its box's contributions (they
// have no tile entries, so the sums are written, not added).
__global__ __launch_bounds__(256) void k_splat_large_bwd(const SplatP *__restrict__ sp, int64_t m,
                                                         RastGeo G, const int *__restrict__ large,
                                                         const int *__restrict__ nlarge,
                                                         const float *__restrict__ g_proj,
                                                         float *__restrict__ acc6) {
    __shared__ float red[4][6];
    const float k2 = G.k * G.k;
    const int n = *nlarge;
    for (int li = blockIdx.x; li < n; li += gridDim.x) {
        const int64_t i = large[li];
        const SplatP P = sp[i];
        const int v = (int)(i / m);
        const int u0 = P.tu0 * RS_T, u1 = min((P.tu1 + 1) * RS_T, G.nu);
        const int v0 = P.tv0 * RS_T, v1 = min((P.tv1 + 1) * RS_T, G.nv);
        const int w = u1 - u0;
        const int64_t npx = (int64_t)w * (v1 - v0);
        float s[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int64_t p = threadIdx.x; p < npx; p += blockDim.x) {
            const int x = u0 + (int)(p % w), y = v0 + (int)(p / w);
            float o[6];
            splat_grad(P, (float)x, (float)y, k2, g_proj[((int64_t)v * G.nv + y) * G.nu + x], o);
#pragma unroll
            for (int q = 0; q < 6; ++q) s[q] += o[q];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) s[q] = wave_sum_lane63(s[q]);
        if ((threadIdx.x & 63) == 63)
#pragma unroll
            for (int q = 0; q < 6; ++q) red[threadIdx.x >> 6][q] = s[q];
        __syncthreads();
        if (threadIdx.x < 6)
            acc6[i * 6 + threadIdx.x] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                        (red[2][threadIdx.x] + red[3][threadIdx.x]);
        __syncthreads();
    }
}

// Chain rule per Gaussian, views in order (double): from the 2-D splat's
// gradients to the mean, scale, quaternion and density.
__global__ __launch_bounds__(256) void k_splat_chain(const float *__restrict__ mean,
                                                     const float *__restrict__ scale,
                                                     const float *__restrict__ quat,
                                                     const float *__restrict__ value, int64_t m,
                                                     int V, RastGeo G,
                                                     const float *__restrict__ angles,
                                                     const float *__restrict__ acc6,
                                                     float *__restrict__ g_mean,
                                                     float *__restrict__ g_scale,
                                                     float *__restrict__ g_quat,
                                                     float *__restrict__ g_value) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m) return;
    double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gv = 0.0;
    for (int v = 0; v < V; ++v) {
        const float *A6 = acc6 + ((int64_t)v * m + g) * 6;
        const double grho = A6[0], gmu[2] = {A6[1], A6[2]}, ga = A6[3], gb = A6[4], gc = A6[5];
        if (grho == 0.0 && gmu[0] == 0.0 && gmu[1] == 0.0 && ga == 0.0 && gb == 0.0 && gc == 0.0)
            continue;
        SplatD D;
        splat_setup(G, (double)angles[v], mean + 3 * g, scale + 3 * g, quat + 4 * g, D);
        if (!D.ok) continue;
        const double rho_hat = (double)value[g] * D.amp;
        gv += grho * D.amp;
        // conic A = Sigma^-1 (entries a, b (twice), c): dL/dSigma^ = -A Gc A
        const double Ai[2][2] = {{D.Sh[2] / D.det2, -D.Sh[1] / D.det2},
                                 {-D.Sh[1] / D.det2, D.Sh[0] / D.det2}};
        const double Gc[2][2] = {{ga, 0.5 * gb}, {0.5 * gb, gc}};
        double T2[2][2], GSh[2][2];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) T2[r][c] = Gc[r][0] * Ai[0][c] + Gc[r][1] * Ai[1][c];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) GSh[r][c] = -(Ai[r][0] * T2[0][c] + Ai[r][1] * T2[1][c]);
        // amplitude: rho^ = rho sqrt(2 pi det3 / det2): d/dSigma~ = rho^/2 Sigma~^-1,
        // d/dSigma^ = -rho^/2 Sigma^-1
        double Sti[3][3];
        {
            const double(*S)[3] = D.St;
            Sti[0][0] = (S[1][1] * S[2][2] - S[1][2] * S[2][1]) / D.det3;
            Sti[0][1] = (S[0][2] * S[2][1] - S[0][1] * S[2][2]) / D.det3;
            Sti[0][2] = (S[0][1] * S[1][2] - S[0][2] * S[1][1]) / D.det3;
            Sti[1][0] = (S[1][2] * S[2][0] - S[1][0] * S[2][2]) / D.det3;
            Sti[1][1] = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) / D.det3;
            Sti[1][2] = (S[0][2] * S[1][0] - S[0][0] * S[1][2]) / D.det3;
            Sti[2][0] = (S[1][0] * S[2][1] - S[1][1] * S[2][0]) / D.det3;
            Sti[2][1] = (S[0][1] * S[2][0] - S[0][0] * S[2][1]) / D.det3;
            Sti[2][2] = (S[0][0] * S[1][1] - S[0][1] * S[1][0]) / D.det3;
        }
        const double hr = 0.5 * grho * rho_hat;
        double GSt[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) GSt[r][c] = hr * Sti[r][c];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) GSt[r][c] += GSh[r][c] - hr * Ai[r][c];
        // Sigma~ = M Sigma M^T: dL/dSigma = M^T G M, dL/dM = 2 G M Sigma
        double GM[3][3], GSig[3][3], MS[3][3], GMM[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                GM[r][c] = GSt[r][0] * D.M[0][c] + GSt[r][1] * D.M[1][c] + GSt[r][2] * D.M[2][c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                GSig[r][c] = D.M[0][r] * GM[0][c] + D.M[1][r] * GM[1][c] + D.M[2][r] * GM[2][c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                MS[r][c] = GM[r][0] * D.Sig[0][c] + GM[r][1] * D.Sig[1][c] + GM[r][2] * D.Sig[2][c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) GMM[r][c] = 2.0 * MS[r][c];
        // M = J W: dL/dJ = dL/dM W^T
        double GJ[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                GJ[r][c] = GMM[r][0] * D.W[c][0] + GMM[r][1] * D.W[c][1] + GMM[r][2] * D.W[c][2];
        // dL/dt: through the centre (rows 0, 1 of J) and through J(t)
        const double su = G.sdd / G.du, sv = G.sdd / G.dv;
        const double tu = D.t[0], tv = D.t[1], td = D.t[2], n = D.nt;
        double gt[3];
        for (int k = 0; k < 3; ++k) gt[k] = D.J[0][k] * gmu[0] + D.J[1][k] * gmu[1];
        gt[2] += GJ[0][0] * (-su / (td * td)) + GJ[1][1] * (-sv / (td * td));
        gt[0] += GJ[0][2] * (-su / (td * td));
        gt[2] += GJ[0][2] * (2.0 * su * tu / (td * td * td));
        gt[1] += GJ[1][2] * (-sv / (td * td));
        gt[2] += GJ[1][2] * (2.0 * sv * tv / (td * td * td));
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k)
                gt[k] += GJ[2][c] * (((c == k) ? 1.0 : 0.0) - D.t[c] * D.t[k] / (n * n)) / n;
        // t = W (p - o): dL/dp = W^T dL/dt
        for (int a = 0; a < 3; ++a) gm[a] += D.W[0][a] * gt[0] + D.W[1][a] * gt[1] + D.W[2][a] * gt[2];
        // Sigma = R diag(s^2) R^T: dL/ds_k = 2 s_k (R^T G R)_kk, dL/dR = 2 G R diag(s^2)
        const double s_[3] = {scale[3 * g], scale[3 * g + 1], scale[3 * g + 2]};
        double GR[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                const double gr = GSig[r][0] * D.R[0][c] + GSig[r][1] * D.R[1][c] + GSig[r][2] * D.R[2][c];
                GR[r][c] = 2.0 * gr * s_[c] * s_[c];
            }
        for (int k = 0; k < 3; ++k) {
            double d = 0.0;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) d += D.R[r][k] * GSig[r][c] * D.R[c][k];
            gs[k] += 2.0 * s_[k] * d;
        }
        const double w = D.qh[0], x = D.qh[1], y = D.qh[2], z = D.qh[3];
        double gqh[4];
        gqh[0] = 2 * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
        gqh[1] = 2 * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2 * x * GR[1][1] - w * GR[1][2] +
                      z * GR[2][0] + w * GR[2][1] - 2 * x * GR[2][2]);
        gqh[2] = 2 * (-2 * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + z * GR[1][2] -
                      w * GR[2][0] + z * GR[2][1] - 2 * y * GR[2][2]);
        gqh[3] = 2 * (-2 * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - 2 * z * GR[1][1] +
                      y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
        const double dot = gqh[0] * w + gqh[1] * x + gqh[2] * y + gqh[3] * z;
        for (int k = 0; k < 4; ++k) gq[k] += (gqh[k] - D.qh[k] * dot) / D.qn;
    }
    for (int a = 0; a < 3; ++a) {
        g_mean[3 * g + a] = (float)gm[a];
        g_scale[3 * g + a] = (float)gs[a];
    }
    for (int k = 0; k < 4; ++k) g_quat[4 * g + k] = (float)gq[k];
    g_value[g] = (float)gv;
}

// ---------------------------------------------------------------- launchers
static RastGeo rast_geo(const pmf_cone_t &c, float k) {
    RastGeo G;
    G.sad = c.sad;
    G.sdd = c.sdd;
    G.du = c.du;
    G.dv = c.dv;
    G.off_u = c.off_u;
    G.off_v = c.off_v;
    G.nu = c.nu;
    G.nv = c.nv;
    G.tiles_u = (c.nu + RS_T - 1) / RS_T;
    G.tiles_v = (c.nv + RS_T - 1) / RS_T;
    G.k = k;
    return G;
}

namespace {
struct RastWs {
    SplatP *sp;
    int *counts, *offsets, *list, *large, *nlarge, *gslot;
    float *acc6, *part;
    size_t total;
};

RastWs rast_ws(void *base, int64_t m, const RastGeo &G, int V) {
    RastWs w;
    const int64_t T = (int64_t)G.tiles_u * G.tiles_v * V;
    const int64_t mv = m * V;
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *r = p ? p + off : nullptr;
        off += align256(bytes);
        return r;
    };
    w.sp = (SplatP *)take(sizeof(SplatP) * (size_t)mv);
    w.counts = (int *)take(sizeof(int) * RS_CSTRIDE * (size_t)T);
    w.offsets = (int *)take(sizeof(int) * (size_t)(T + 1));
    w.list = (int *)take(sizeof(int) * (size_t)mv * RS_TMAX);
    w.large = (int *)take(sizeof(int) * (size_t)mv);
    w.nlarge = (int *)take(sizeof(int));
    w.acc6 = (float *)take(sizeof(float) * 6 * (size_t)mv);
    w.gslot = (int *)take(sizeof(int) * (size_t)mv * RS_TMAX);
    w.part = (float *)take(sizeof(float) * 6 * (size_t)mv * RS_TMAX);
    w.total = off;
    return w;
}
}  // namespace

size_t rasterize_workspace(int64_t m, const pmf_cone_t &c, int V) {
    return rast_ws(nullptr, m, rast_geo(c, 3.0f), V).total;
}

static hipError_t rast_bin(const pmf_gauss_t &gs, const RastGeo &G, const float *angles, int V,
                           const RastWs &w, hipStream_t s) {
    const int64_t T = (int64_t)G.tiles_u * G.tiles_v * V;
    const int64_t mv = gs.m * V;
    hipError_t e;
    if ((e = launch_fill_i32(w.counts, RS_CSTRIDE * T, 0, s)) != hipSuccess) return e;
    if ((e = launch_fill_i32(w.nlarge, 1, 0, s)) != hipSuccess) return e;
    {
        ProfScope prof_("rasterize_bin", s);
        k_splat_prep<<<(unsigned)((mv + 255) / 256), 256, 0, s>>>(gs.mean, gs.scale, gs.quat,
                                                                  gs.value, gs.m, V, G, angles,
                                                                  w.sp, w.counts, w.gslot, w.large,
                                                                  w.nlarge);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_rast_scan<<<1, 1024, 0, s>>>(w.counts, T, w.offsets);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_splat_fill<<<(unsigned)((mv + 255) / 256), 256, 0, s>>>(w.sp, gs.m, V, G, w.offsets,
                                                                  w.list, w.gslot);
    }
    return hipGetLastError();
}

hipError_t launch_rasterize(const pmf_gauss_t &gs, const pmf_cone_t &c, const float *angles,
                            int V, float k, float *proj, void *ws, hipStream_t s) {
    const RastGeo G = rast_geo(c, k);
    const RastWs w = rast_ws(ws, gs.m, G, V);
    hipError_t e = rast_bin(gs, G, angles, V, w, s);
    if (e != hipSuccess) return e;
    const int64_t T = (int64_t)G.tiles_u * G.tiles_v * V;
    {
        ProfScope prof_("rasterize", s);
        k_splat_fwd<<<(unsigned)T, RS_THREADS, 0, s>>>(w.sp, gs.m, G, w.offsets, w.list, w.large,
                                                        w.nlarge, proj);
    }
    return hipGetLastError();
}

// rebin = false: ws already holds the binning of a pmf_rasterize call on the
// same inputs (splat records, tile lists, list positions), which is reused.
hipError_t launch_rasterize_bwd(const pmf_gauss_t &gs, const pmf_cone_t &c, const float *angles,
                                int V, float k, const float *g_proj, const pmf_gauss_grad_t &gg,
                                void *ws, hipStream_t s, bool rebin) {
    const RastGeo G = rast_geo(c, k);
    const RastWs w = rast_ws(ws, gs.m, G, V);
    hipError_t e = rebin ? rast_bin(gs, G, angles, V, w, s) : hipSuccess;
    if (e != hipSuccess) return e;
    const int64_t T = (int64_t)G.tiles_u * G.tiles_v * V;
    const int64_t mv = gs.m * V;
    {
        ProfScope prof_("rasterize_bwd", s);
        k_splat_bwd<<<dim3((unsigned)T, RB_SPLIT), RS_THREADS, 0, s>>>(w.sp, G, w.offsets, w.list,
                                                                      g_proj, w.part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (mv > 0) {
            k_splat_gather<<<(unsigned)((mv + 255) / 256), 256, 0, s>>>(w.sp, mv, w.gslot, w.part,
                                                                        w.acc6);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        k_splat_large_bwd<<<1024, 256, 0, s>>>(w.sp, gs.m, G, w.large, w.nlarge, g_proj, w.acc6);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_splat_chain<<<(unsigned)((gs.m + 255) / 256), 256, 0, s>>>(
            gs.mean, gs.scale, gs.quat, gs.value, gs.m, V, G, angles, w.acc6, gg.mean, gg.scale,
            gg.quat, gg.value);
    }
    return hipGetLastError();
}

}  // namespace pmf
