// fused.hip -- the motion path of all views in one pass (batched form).
//
// Forward: one thread per voxel samples the L*B*3 basis values once, then for
// every view forms the DVF in registers (Eq. 3) and warps the reference
// volume (Eq. 2); only the warped volumes reach memory, and one launch
// projects all of them.
//
// Adjoint: the back-projection of every view's residual (brick owner, LDS),
// then one pass over the voxels that, for every view, recomputes the DVF,
// takes the warp adjoint and the Eq. 3 adjoint in registers:
//   - g_ref: added into an LDS copy of the brick plus a halo in fixed point,
//     staged per brick and gathered in a fixed order; the rare displacement
//     that leaves the halo adds into a 64-bit fixed-point copy of g_ref with
//     integer atomics, so the sums do not depend on their order;
//   - dL/dE: sum over views of coeff * g_dvf, per voxel in registers; stored
//     directly for a level on the output grid, otherwise handed to the
//     separable upsampling transpose;
//   - dL/dcoeff: per-view wave sums into LDS, then per-workgroup partials
//     summed in block order.
#include <math.h>

#include <algorithm>

#include "pmf_internal.h"

namespace pmf {

// One scan's share of a ragged launch: workgroups [first[k], first[k+1])
// belong to scan k.
struct CWK {
    const float *ref;
    GridK g;
    LevelsK lv;
    const float *coeff;
    int V;
    float *warped;
    int items;              // workgroups of 256 voxels
};
struct CWTab {
    CWK s[MAXS];
    int first[MAXS + 1];
    int n;
};

// Trilinear read of a y-paired volume (element (i, j, k) holds V[i][j][k] and
// V[i][j+1][k]) at voxel (x0, x1, x2) displaced by (t0, t1, t2) voxels: two
// 16-byte loads, the same cell, blend and order as sample_disp, 0 outside the
// box.
__device__ __forceinline__ float sample_disp_paired(const float *__restrict__ vp, const int n[3],
                                                    int x0, int x1, int x2, float t0, float t1,
                                                    float t2) {
    int i0, i1, i2;
    float f0, f1, f2;
    if (!disp_cell(x0, t0, n[0], i0, f0) || !disp_cell(x1, t1, n[1], i1, f1) ||
        !disp_cell(x2, t2, n[2], i2, f2))
        return 0.0f;
    const float *pa = vp + 2 * ((i0 * n[1] + i1) * n[2] + i2);
    const float *pd = pa + 2 * n[1] * n[2];
    const float a0 = pa[0], a1 = pa[1], a2 = pa[2], a3 = pa[3];
    const float d0 = pd[0], d1 = pd[1], d2 = pd[2], d3 = pd[3];
    const float c00 = lerp1(a0, a2, f2), c01 = lerp1(a1, a3, f2);
    const float c10 = lerp1(d0, d2, f2), c11 = lerp1(d1, d3, f2);
    return lerp1(lerp1(c00, c01, f1), lerp1(c10, c11, f1), f0);
}

// y-paired copy of a volume: out[2j] = V[j], out[2j+1] = V[j + n2] (0 on the
// last row, which no trilinear read takes).
__global__ __launch_bounds__(256) void k_pair_volume(const float *__restrict__ in, GridK g,
                                                     float2 *__restrict__ out) {
    const int64_t N = grid_size(g);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int iy = (int)((j / g.n[2]) % g.n[1]);
    out[j] = make_float2(in[j], iy + 1 < g.n[1] ? in[j + g.n[2]] : 0.0f);
}

// Body of one voxel; the restrict-qualified parameters (kept through
// inlining) let the per-view coefficients come through scalar loads.  With
// PAIRED the warped volumes are written in the y-paired layout the
// projection reads (two floats per voxel: its value and the next row's).
template <int L, int B, bool PAIRED>
__device__ __forceinline__ void combine_warp_voxel(const float *__restrict__ ref, const GridK &g,
                                                   const LevelsK &lv,
                                                   const float *__restrict__ coeff, int V,
                                                   float *__restrict__ warped, int64_t j) {
    const int64_t N = grid_size(g);
    if (j >= N) return;
    const int iz = (int)(j % g.n[2]);
    const int iy = (int)((j / g.n[2]) % g.n[1]);
    const int ix = (int)(j / ((int64_t)g.n[2] * g.n[1]));
    float sv[L][B][3];
    basis_samples<L, B>(lv, ix, iy, iz, sv);
    for (int v = 0; v < V; ++v) {
        const float *cv = coeff + (int64_t)v * L * B * 3;
        float d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float t = 0.0f;
#pragma unroll
            for (int l = 0; l < L; ++l)
#pragma unroll
                for (int b = 0; b < B; ++b) t = fmaf(cv[(l * B + b) * 3 + k], sv[l][b][k], t);
            d[k] = t;
        }
        // the sample point in voxel units is (ix, iy, iz) + d / h
        const float t0 = d[0] * g.inv_h[0], t1 = d[1] * g.inv_h[1], t2 = d[2] * g.inv_h[2];
        // with PAIRED, ref is the y-paired copy of the reference volume
        const float val = PAIRED ? sample_disp_paired(ref, g.n, ix, iy, iz, t0, t1, t2)
                                 : sample_disp(ref, g.n, ix, iy, iz, t0, t1, t2);
        if (PAIRED) {
            // y-paired layout: this voxel is the first of its own pair and the
            // second of the pair that starts one row below
            float *w = warped + (int64_t)v * 2 * N + 2 * j;
            w[0] = val;
            if (iy > 0) w[1 - 2 * (int64_t)g.n[2]] = val;
        } else {
            warped[(int64_t)v * N + j] = val;
        }
    }
}

template <int L, int B, bool PAIRED>
__global__ __launch_bounds__(256) void k_combine_warp(CWTab t) {
    const int job = job_of(t, (int)blockIdx.x);
    const CWK &cj = t.s[job];
    const int item = job_item(t, job, (int)blockIdx.x);
    if (item >= cj.items) return;
    const int64_t j = (int64_t)item * blockDim.x + threadIdx.x;
    combine_warp_voxel<L, B, PAIRED>(cj.ref, cj.g, cj.lv, cj.coeff, cj.V, cj.warped, j);
}



// Brick of the adjoint pass: 8x8x8 voxels, one per thread; LDS box with a
// halo of HALO voxels on every side for the g_ref scatter.  Views are taken
// in chunks of at most VCH per launch.
constexpr int FB = 8;
constexpr int HALO = 3;
constexpr int HB = FB + 2 * HALO + 1;
constexpr int HB3 = HB * HB * HB;
constexpr int VCH = 64;
constexpr int FLUSH = 32;  // views per fixed-point accumulation round
constexpr int WB_THREADS = FB * FB * FB;    // one voxel per thread
constexpr int WB_WAVES = WB_THREADS / 64;
constexpr int LO_BITS = 17; // 512 * FLUSH * 2^(LO_BITS-1) < 2^31

struct GOut {
    float *dst[MAXL];   // per level: [3B][N] destination (g_bases or staging buffer)
};

// Warp adjoint and Eq. 3 adjoint of one 8^3 brick for a chunk of views.
// dL/dI_ref is scattered into an LDS box (brick + halo) in fixed point with
// integer LDS atomics: per round of up to FLUSH views the scale is
// 2^30 / (512 * views * M) with M the largest |dL/dI_v| of those views, which
// bounds every partial sum; each scaled contribution is split into its
// nearest integer (high word) and the remainder times 2^LO_BITS (low word),
// so the two 32-bit sums keep about 47 bits; each round is folded into a
// float box.
// The float box is staged per brick and summed by k_gather_boxes;
// displacements that leave the halo add into a 64-bit fixed-point volume
// (fix_add, scale from the largest |dL/dI_v| of all views), which the last
// k_gather_boxes folds in.  dL/dw of
// each view is reduced over a wave, written to that wave's LDS slot, and the
// slots are summed over the waves in a fixed order into the brick's partials
// (reduced over bricks by k_reduce_coeff_parts / _final), so it is deterministic.
struct WCK {
    const float *ref;       // y-paired when paired (see k_pair_volume)
    int paired;
    GridK g;
    LevelsK lv;
    const float *coeff;     // this chunk's first view
    int V;                  // views in this chunk
    const float *g_I;
    const unsigned *vmax;
    const unsigned *vmax_all;   // largest |dL/dI_v| over every view of the scan
    long long *fix;             // [N] 64-bit fixed point for the halo overflow
    float *stage;
    GOut gout;
    int accumulate;
    int nb1, nb2;
    float *partial;
    int items;              // bricks
};
struct WCTab {
    WCK s[MAXS];
    int first[MAXS + 1];
    int n;
};

template <int L, int B>
__device__ __forceinline__ void warp_combine_bwd_brick(
    const float *__restrict__ ref, int paired, const GridK &g, const LevelsK &lv,
    const float *__restrict__ coeff, int V, const float *__restrict__ g_I,
    const unsigned *__restrict__ vmax, const unsigned *__restrict__ vmax_all,
    long long *__restrict__ fix, float *__restrict__ stage, const GOut &gout, int accumulate,
    int nb1, int nb2, float *__restrict__ partial, int blk) {
    constexpr int NC = L * B * 3;
    extern __shared__ float smem[];
    int *ibox = (int *)smem;              // HB^3 fixed point, high words
    int *lbox = (int *)smem + HB3;        // HB^3 fixed point, low words
    float *fbox = smem + 2 * HB3;         // HB^3 float
    float *wslot = smem + 3 * HB3;        // [WB_WAVES][FLUSH][NC]: each wave's dL/dw of a round
    for (int i = threadIdx.x; i < HB3; i += WB_THREADS) {
        ibox[i] = 0;
        lbox[i] = 0;
        fbox[i] = 0.0f;
    }
    const int bid = blk;
    const int b2 = bid % nb2, b1 = (bid / nb2) % nb1, b0 = bid / (nb2 * nb1);
    const int B0 = b0 * FB, B1 = b1 * FB, B2 = b2 * FB;
    const int64_t N = grid_size(g);
    const int s1 = g.n[2], s0 = g.n[1] * g.n[2];

    // one voxel per thread
    const int t = threadIdx.x;
    const int vx = B0 + t / (FB * FB), vy = B1 + (t / FB) % FB, vz = B2 + t % FB;
    const bool ok = vx < g.n[0] && vy < g.n[1] && vz < g.n[2];
    const int64_t jj = ok ? ((int64_t)vx * g.n[1] + vy) * g.n[2] + vz : 0;
    float sv[L][B][3];
    basis_samples<L, B>(lv, ok ? vx : 0, ok ? vy : 0, ok ? vz : 0, sv);
    float G[L][B][3];
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) G[l][b][k] = 0.0f;
    __syncthreads();

    const int lane = t & 63, wave = t >> 6;
    const double fscale = fix_scale(*vmax_all);
    for (int r0 = 0; r0 < V; r0 += FLUSH) {
        const int r1 = min(V, r0 + FLUSH);
        float M = 0.0f;
        for (int v = r0; v < r1; ++v) M = fmaxf(M, __uint_as_float(vmax[v]));
        const float scale = M > 0.0f ? 1073741824.0f / (512.0f * (float)(r1 - r0) * M) : 0.0f;
        for (int v = r0; v < r1; ++v) {
            const float *cv = coeff + (int64_t)v * L * B * 3;
            float gD[3] = {0.0f, 0.0f, 0.0f};
            do {
                if (!ok) break;
                float d[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float acc = 0.0f;
#pragma unroll
                    for (int l = 0; l < L; ++l)
#pragma unroll
                        for (int b = 0; b < B; ++b)
                            acc = fmaf(cv[(l * B + b) * 3 + k], sv[l][b][k], acc);
                    d[k] = acc;
                }
                const float t0 = d[0] * g.inv_h[0], t1 = d[1] * g.inv_h[1],
                            t2 = d[2] * g.inv_h[2];
                int i0, i1, i2;
                float f0, f1, f2;
                if (!disp_cell(vx, t0, g.n[0], i0, f0) || !disp_cell(vy, t1, g.n[1], i1, f1) ||
                    !disp_cell(vz, t2, g.n[2], i2, f2))
                    break;
                const float go = g_I[(int64_t)v * N + jj];
                if (go == 0.0f) break;
                const int64_t base = ((int64_t)i0 * g.n[1] + i1) * g.n[2] + i2;
                float c000, c001, c010, c011, c100, c101, c110, c111;
                if (paired) {
                    // the 2x2 (y, z) corners of a cell are 16 contiguous
                    // (8-byte aligned) bytes: one load each for x and x+1
                    typedef float v4a8 __attribute__((ext_vector_type(4), aligned(8)));
                    const float *pa = ref + 2 * base;
                    const v4a8 a = *(const v4a8 *)pa, e = *(const v4a8 *)(pa + 2 * (int64_t)s0);
                    c000 = a.x; c010 = a.y; c001 = a.z; c011 = a.w;
                    c100 = e.x; c110 = e.y; c101 = e.z; c111 = e.w;
                } else {
                    const float *p = ref + base;
                    c000 = p[0]; c001 = p[1]; c010 = p[s1]; c011 = p[s1 + 1];
                    c100 = p[s0]; c101 = p[s0 + 1]; c110 = p[s0 + s1]; c111 = p[s0 + s1 + 1];
                }
                const float a00 = lerp1(c000, c001, f2), a01 = lerp1(c010, c011, f2);
                const float a10 = lerp1(c100, c101, f2), a11 = lerp1(c110, c111, f2);
                const float ddx = lerp1(a10, a11, f1) - lerp1(a00, a01, f1);
                const float ddy = lerp1(a01, a11, f0) - lerp1(a00, a10, f0);
                const float e00 = lerp1(c000, c010, f1), e01 = lerp1(c001, c011, f1);
                const float e10 = lerp1(c100, c110, f1), e11 = lerp1(c101, c111, f1);
                const float ddz = lerp1(e01, e11, f0) - lerp1(e00, e10, f0);
                gD[0] = go * ddx * g.inv_h[0] * disp_free(vx, t0, g.n[0]);
                gD[1] = go * ddy * g.inv_h[1] * disp_free(vy, t1, g.n[1]);
                gD[2] = go * ddz * g.inv_h[2] * disp_free(vz, t2, g.n[2]);
                const int l0 = i0 - (B0 - HALO), l1 = i1 - (B1 - HALO), l2 = i2 - (B2 - HALO);
                const bool inbox = l0 >= 0 && l0 + 1 < HB && l1 >= 0 && l1 + 1 < HB && l2 >= 0 &&
                                   l2 + 1 < HB;
                if (inbox) {
                    const float gs = go * scale;
                    const float wx0 = gs * (1.0f - f0), wx1 = gs * f0;
                    const float q00 = wx0 * (1.0f - f1), q01 = wx0 * f1;
                    const float q10 = wx1 * (1.0f - f1), q11 = wx1 * f1;
                    const float g2 = 1.0f - f2;
                    const int o = (l0 * HB + l1) * HB + l2;
                    const float cw[8] = {q00 * g2, q00 * f2, q01 * g2, q01 * f2,
                                         q10 * g2, q10 * f2, q11 * g2, q11 * f2};
                    const int off[8] = {0, 1, HB, HB + 1, HB * HB, HB * HB + 1, HB * HB + HB,
                                        HB * HB + HB + 1};
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const float hi = rintf(cw[k]);
                        atomicAdd(ibox + o + off[k], (int)hi);
                        atomicAdd(lbox + o + off[k], __float2int_rn((cw[k] - hi) * (float)(1 << LO_BITS)));
                    }
                } else {
                    const float w0[2] = {1.0f - f0, f0}, w1[2] = {1.0f - f1, f1},
                                w2[2] = {1.0f - f2, f2};
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
#pragma unroll
                            for (int c = 0; c < 2; ++c)
                                fix_add(&fix[base + a * s0 + b * s1 + c],
                                        (double)(go * w0[a] * w1[b] * w2[c]), fscale);
                }
            } while (false);
            // dL/dE: per voxel over views; dL/dw[v]: per-lane products,
            // reduce-scattered over the wave in groups of 16 coefficients
            // into this wave's slot (summed over the waves in a fixed order
            // at the end of the round)
#pragma unroll
            for (int l = 0; l < L; ++l)
#pragma unroll
                for (int b = 0; b < B; ++b)
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        G[l][b][k] = fmaf(cv[(l * B + b) * 3 + k], gD[k], G[l][b][k]);
            float *slot = wslot + (wave * FLUSH + (v - r0)) * NC;
#pragma unroll
            for (int g0 = 0; g0 < NC; g0 += 16) {
                float x[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int ci = g0 + q;
                    const int k = ci % 3, lb = ci / 3;
                    x[q] = ci < NC ? gD[k] * sv[lb / B][lb % B][k] : 0.0f;
                }
                const float tot = wave_reduce_scatter16(x, lane);
                const int ci = g0 + scatter16_index(lane);
                if ((lane & 3) == 0 && ci < NC) slot[ci] = tot;
            }
        }
        __syncthreads();
        if (scale > 0.0f) {
            const float inv = 1.0f / scale;
            for (int i = t; i < HB3; i += WB_THREADS) {
                const int a = ibox[i], u = lbox[i];
                if (a | u) {
                    fbox[i] += ((float)a + (float)u * (1.0f / (float)(1 << LO_BITS))) * inv;
                    ibox[i] = 0;
                    lbox[i] = 0;
                }
            }
        }
        for (int i = t; i < (r1 - r0) * NC; i += WB_THREADS) {
            float sum = 0.0f;
#pragma unroll
            for (int w = 0; w < WB_WAVES; ++w) sum += wslot[w * FLUSH * NC + i];
            partial[((int64_t)blk * V + r0) * NC + i] = sum;
        }
        __syncthreads();
    }
    float *st = stage + (int64_t)blk * HB3;
    for (int i = t; i < HB3; i += WB_THREADS) st[i] = fbox[i];
    if (ok) {
#pragma unroll
        for (int l = 0; l < L; ++l)
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    float *dst = gout.dst[l] + (int64_t)(b * 3 + k) * N + jj;
                    *dst = accumulate ? *dst + G[l][b][k] : G[l][b][k];
                }
    }
}

template <int L, int B>
__global__ __launch_bounds__(WB_THREADS) void k_warp_combine_bwd(WCTab t) {
    const int job = job_of(t, (int)blockIdx.x);
    const WCK &wj = t.s[job];
    const int item = job_item(t, job, (int)blockIdx.x);
    if (item >= wj.items) return;
    warp_combine_bwd_brick<L, B>(wj.ref, wj.paired, wj.g, wj.lv, wj.coeff, wj.V, wj.g_I, wj.vmax,
                                 wj.vmax_all, wj.fix, wj.stage, wj.gout, wj.accumulate, wj.nb1,
                                 wj.nb2, wj.partial, item);
}

// g_ref[p] += sum of the staged boxes that cover voxel p (at most 2 bricks
// per axis), in a fixed order, plus (when fix is given: the last chunk of
// views) the 64-bit fixed-point halo overflow.
__global__ __launch_bounds__(256) void k_gather_boxes(const float *__restrict__ stage, GridK g,
                                                      int nb0, int nb1, int nb2,
                                                      const long long *__restrict__ fix,
                                                      const unsigned *__restrict__ vmax_all,
                                                      float *__restrict__ g_ref) {
    // N < 2^31 (checked on the host): 32-bit index arithmetic
    const unsigned N = (unsigned)grid_size(g);
    const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const unsigned q = j / (unsigned)g.n[2];
    const int p2 = (int)(j - q * (unsigned)g.n[2]);
    const int p0 = (int)(q / (unsigned)g.n[1]);
    const int p1 = (int)(q - (unsigned)p0 * (unsigned)g.n[1]);
    // bricks b with b*FB - HALO <= p <= b*FB + FB + HALO
    const int a0 = max(0, (p0 - FB - HALO + FB - 1) / FB), e0 = min(nb0 - 1, (p0 + HALO) / FB);
    const int a1 = max(0, (p1 - FB - HALO + FB - 1) / FB), e1 = min(nb1 - 1, (p1 + HALO) / FB);
    const int a2 = max(0, (p2 - FB - HALO + FB - 1) / FB), e2 = min(nb2 - 1, (p2 + HALO) / FB);
    float s = 0.0f;
    for (int b0 = a0; b0 <= e0; ++b0)
        for (int b1 = a1; b1 <= e1; ++b1)
            for (int b2 = a2; b2 <= e2; ++b2) {
                const int l0 = p0 - (b0 * FB - HALO), l1 = p1 - (b1 * FB - HALO),
                          l2 = p2 - (b2 * FB - HALO);
                s += stage[((int64_t)(b0 * nb1 + b1) * nb2 + b2) * HB3 + (l0 * HB + l1) * HB + l2];
            }
    if (fix) {
        const long long fv = fix[j];
        if (fv != 0) s += (float)((double)fv / fix_scale(*vmax_all));  // nonzero: scale > 0
    }
    g_ref[j] += s;
}

// g_coeff[v0 + v][...] = sum over bricks of the per-brick partials
// ([brick][v][c], vnc = views x channels per brick), in two fixed-order
// stages: P contiguous brick ranges summed for every output with coalesced
// reads, then the P range sums of each output in a fixed tree.
__global__ __launch_bounds__(256) void k_reduce_coeff_parts(const float *__restrict__ partial,
                                                            int nblk, int vnc, int P,
                                                            float *__restrict__ part2) {
    const int p = blockIdx.y, o = blockIdx.x * 256 + threadIdx.x;
    if (o >= vnc) return;
    const int b0 = (int)((int64_t)nblk * p / P), b1 = (int)((int64_t)nblk * (p + 1) / P);
    float s = 0.0f;
    for (int i = b0; i < b1; ++i) s += partial[(int64_t)i * vnc + o];
    part2[(int64_t)p * vnc + o] = s;
}

// one workgroup per output: its P (<= 256) range sums, one per thread, in a
// fixed tree
__global__ __launch_bounds__(256) void k_reduce_coeff_final(const float *__restrict__ part2, int P,
                                                            int vnc, float *__restrict__ g_coeff) {
    __shared__ float red[4];
    const int o = blockIdx.x;
    float s = (int)threadIdx.x < P ? part2[(int64_t)threadIdx.x * vnc + o] : 0.0f;
    s = wave_sum_lane63(s);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) g_coeff[o] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The warped volumes go to the workspace in the y-paired layout when the
// projection's 32-bit byte offsets and 24-bit strides still hold for it
// (2 N floats < 2^32 bytes, 2 n1 n2 < 2^24).
static bool use_paired(const GridK &g) {
    return grid_size(g) * 8 < ((int64_t)1 << 32) &&
           2 * (int64_t)g.n[1] * g.n[2] < ((int64_t)1 << 24);
}

// Workspace: the warped volumes (y-paired when possible), then the y-paired
// copy of the reference volume.
size_t warp_project_workspace(const LevelsK &lv, int V, const GridK &g, const pmf_cone_t &c) {
    (void)lv;
    (void)c;
    const size_t N = (size_t)grid_size(g);
    return use_paired(g) ? align256(sizeof(float) * N * V * 2) + align256(sizeof(float) * N * 2)
                         : align256(sizeof(float) * N * V);
}

// Forward of the motion path for a ragged batch: one combine+warp launch and
// one projection launch over every scan's voxels / tiles.
hipError_t launch_warp_project_jobs(const WPJob *jobs, int n, hipStream_t s) {
    if (n < 1 || n > MAXS) return hipErrorInvalidValue;
    const int L = jobs[0].lv.L, Bb = jobs[0].lv.B;
    CWTab t{};
    t.n = n;
    ProjJob pj[MAXS];
    bool paired = true;
    for (int k = 0; k < n; ++k) paired = paired && use_paired(jobs[k].g);
    for (int k = 0; k < n; ++k) {
        const WPJob &j = jobs[k];
        if (j.lv.L != L || j.lv.B != Bb) return hipErrorInvalidValue;
        const int64_t N = grid_size(j.g);
        CWK &c = t.s[k];
        c.ref = j.ref;
        if (paired) {
            // y-paired copy of the reference volume after the warped volumes
            float2 *rp = (float2 *)((char *)j.ws + align256(sizeof(float) * (size_t)N * j.V * 2));
            {
                ProfScope prof_("pair_volume", s);
                k_pair_volume<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(j.ref, j.g, rp);
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            c.ref = (const float *)rp;
        }
        c.g = j.g;
        c.lv = j.lv;
        c.coeff = j.coeff;
        c.V = j.V;
        c.warped = (float *)j.ws;
        c.items = (int)((N + 255) / 256);
        t.first[k + 1] = t.first[k] + align8(c.items);
        pj[k] = ProjJob{c.warped, paired ? 2 * N : N, j.g, j.c, j.angles, j.V, j.proj, paired};
    }
    for (int k = n + 1; k <= MAXS; ++k) t.first[k] = t.first[n];
    hipError_t e = dispatch_lb(L, Bb, [&](auto Lc, auto Bc) {
        constexpr int LL = decltype(Lc)::value, BB = decltype(Bc)::value;
        {
            ProfScope prof_("combine_warp", s);
            if (paired)
                k_combine_warp<LL, BB, true><<<(unsigned)t.first[n], 256, 0, s>>>(t);
            else
                k_combine_warp<LL, BB, false><<<(unsigned)t.first[n], 256, 0, s>>>(t);
        }
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return launch_project_jobs(pj, n, s);
}

hipError_t launch_warp_project(const float *ref, const GridK &g, const LevelsK &lv,
                               const float *coeff, int V, const ConeK &c, const float *angles,
                               float *proj, void *ws, hipStream_t s) {
    WPJob j;
    j.ref = ref;
    j.g = g;
    j.lv = lv;
    j.coeff = coeff;
    j.V = V;
    j.c = c;
    j.angles = angles;
    j.proj = proj;
    j.ws = ws;
    return launch_warp_project_jobs(&j, 1, s);
}

struct BwdLayout {
    size_t gI, rays, gbuf, partial, stage, vmax, fix, pref, adj, total;
    int nbrick, nb[3];
};

static BwdLayout bwd_layout(const LevelsK &lv, const GridK *lvl_grids, int V, const GridK &g,
                            int nu, int nv) {
    BwdLayout b;
    const int64_t N = grid_size(g);
    for (int a = 0; a < 3; ++a) b.nb[a] = (g.n[a] + FB - 1) / FB;
    b.nbrick = b.nb[0] * b.nb[1] * b.nb[2];
    size_t adj = 0;
    int ncoarse = 0;
    for (int l = 0; l < lv.L; ++l) {
        const AxisMap &m = lv.map[l];
        if (m.ident[0] && m.ident[1] && m.ident[2]) continue;
        ++ncoarse;
        size_t w = upsample_adjoint_workspace(3 * lv.B, lvl_grids[l], g, m);
        if (w > adj) adj = w;
    }
    pmf_cone_t pc{};
    pc.nu = nu;
    pc.nv = nv;
    const int vc = V < VCH ? V : VCH;
    b.gI = align256(sizeof(float) * (size_t)N * V);
    b.rays = project_bwd_workspace(g, pc, V);
    b.gbuf = align256(sizeof(float) * (size_t)N * 3 * lv.B * (size_t)ncoarse);
    b.partial = align256(sizeof(float) * (size_t)b.nbrick * vc * lv.L * lv.B * 3);
    b.stage = align256(sizeof(float) * (size_t)b.nbrick * HB3);
    b.vmax = align256(sizeof(unsigned) * ((size_t)V + 1));    // per view, then over all views
    b.fix = align256(sizeof(long long) * (size_t)N);
    b.pref = use_paired(g) ? align256(sizeof(float) * 2 * (size_t)N) : 0;
    b.adj = adj;
    b.total = b.gI + b.rays + b.gbuf + b.partial + b.stage + b.vmax + b.fix + b.pref + b.adj;
    return b;
}

size_t warp_project_bwd_workspace(const LevelsK &lv, const GridK *lvl_grids, int V, const GridK &g,
                                  const pmf_cone_t &c) {
    return bwd_layout(lv, lvl_grids, V, g, c.nu, c.nv).total;
}

namespace {
// One scan's pieces of the adjoint workspace.
struct BwdScan {
    BwdLayout lay;
    float *gI, *gbuf, *partial, *stage;
    float2 *pref;           // y-paired reference volume, or null
    void *rays, *adjws;
    unsigned *vmax;         // [V + 1]: per view, then the largest
    long long *fix;         // [N]
    GOut gout;
    const float *staged[MAXL];
};

BwdScan bwd_scan(const WPBJob &j) {
    BwdScan b;
    b.lay = bwd_layout(j.lv, j.lvl_grids, j.V, j.g, j.c.nu, j.c.nv);
    char *w = (char *)j.ws;
    b.gI = (float *)w;
    w += b.lay.gI;
    b.rays = w;
    w += b.lay.rays;
    b.gbuf = (float *)w;
    w += b.lay.gbuf;
    b.partial = (float *)w;
    w += b.lay.partial;
    b.stage = (float *)w;
    w += b.lay.stage;
    b.vmax = (unsigned *)w;
    w += b.lay.vmax;
    b.fix = (long long *)w;
    w += b.lay.fix;
    b.pref = b.lay.pref ? (float2 *)w : nullptr;
    w += b.lay.pref;
    b.adjws = w;
    const int64_t N = grid_size(j.g);
    int nst = 0;
    for (int l = 0; l < MAXL; ++l) {
        b.gout.dst[l] = nullptr;
        b.staged[l] = nullptr;
    }
    for (int l = 0; l < j.lv.L; ++l) {
        const AxisMap &m = j.lv.map[l];
        if (m.ident[0] && m.ident[1] && m.ident[2]) {
            b.gout.dst[l] = j.g_bases[l];
        } else {
            b.gout.dst[l] = b.gbuf + (int64_t)(nst++) * N * 3 * j.lv.B;
            b.staged[l] = b.gout.dst[l];
        }
    }
    return b;
}
}  // namespace

// Adjoint of the motion path for a ragged batch: one back-projection launch
// and, per chunk of up to VCH views, one warp/combine adjoint launch over
// every scan's bricks; the small per-scan reductions follow.
hipError_t launch_warp_project_bwd_jobs(const WPBJob *jobs, int n, hipStream_t s) {
    if (n < 1 || n > MAXS) return hipErrorInvalidValue;
    const int L = jobs[0].lv.L, Bb = jobs[0].lv.B;
    const int NC = L * Bb * 3;
    BwdScan sc[MAXS];
    BwdJob bj[MAXS];
    int vmax_views = 0;
    hipError_t e;
    for (int k = 0; k < n; ++k) {
        const WPBJob &j = jobs[k];
        if (j.lv.L != L || j.lv.B != Bb) return hipErrorInvalidValue;
        sc[k] = bwd_scan(j);
        if ((e = launch_fill_i32((int32_t *)sc[k].vmax, j.V, 0, s)) != hipSuccess) return e;
        bj[k] = BwdJob{j.g_proj, j.g, j.c, j.angles, j.V, sc[k].gI, grid_size(j.g), sc[k].rays,
                       sc[k].vmax};
        if (j.V > vmax_views) vmax_views = j.V;
    }
    if ((e = launch_project_bwd_jobs(bj, n, s)) != hipSuccess) return e;
    for (int k = 0; k < n; ++k) {
        const WPBJob &j = jobs[k];
        if ((e = launch_fill(j.g_ref, grid_size(j.g), 0.0f, s)) != hipSuccess) return e;
        if ((e = launch_max_u32(sc[k].vmax, j.V, sc[k].vmax + j.V, s)) != hipSuccess) return e;
        if ((e = launch_fill_i32((int32_t *)sc[k].fix, 2 * grid_size(j.g), 0, s)) != hipSuccess)
            return e;
        if (sc[k].pref) {
            const int64_t N = grid_size(j.g);
            {
                ProfScope prof_("pair_volume", s);
                k_pair_volume<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(j.ref, j.g, sc[k].pref);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    for (int v0 = 0; v0 < vmax_views; v0 += VCH) {
        WCTab t{};
        int idx[MAXS];
        int vcs[MAXS];
        for (int k = 0; k < n; ++k) {
            const WPBJob &j = jobs[k];
            if (j.V <= v0) continue;
            const int vc = j.V - v0 < VCH ? j.V - v0 : VCH;
            const int64_t N = grid_size(j.g);
            WCK &w = t.s[t.n];
            w.ref = sc[k].pref ? (const float *)sc[k].pref : j.ref;
            w.paired = sc[k].pref != nullptr;
            w.g = j.g;
            w.lv = j.lv;
            w.coeff = j.coeff + (int64_t)v0 * NC;
            w.V = vc;
            w.g_I = sc[k].gI + (int64_t)v0 * N;
            w.vmax = sc[k].vmax + v0;
            w.vmax_all = sc[k].vmax + j.V;
            w.fix = sc[k].fix;
            w.stage = sc[k].stage;
            w.gout = sc[k].gout;
            w.accumulate = v0 > 0;
            w.nb1 = sc[k].lay.nb[1];
            w.nb2 = sc[k].lay.nb[2];
            w.partial = sc[k].partial;
            w.items = sc[k].lay.nbrick;
            t.first[t.n + 1] = t.first[t.n] + align8(w.items);
            idx[t.n] = k;
            vcs[t.n] = vc;
            ++t.n;
        }
        for (int k = t.n + 1; k <= MAXS; ++k) t.first[k] = t.first[t.n];
        const size_t lds = sizeof(float) * (3 * (size_t)HB3 + (size_t)WB_WAVES * FLUSH * NC);
        e = dispatch_lb(L, Bb, [&](auto Lc, auto Bc) {
            constexpr int LL = decltype(Lc)::value, BB = decltype(Bc)::value;
            {
                ProfScope prof_("warp_combine_bwd", s);
                k_warp_combine_bwd<LL, BB><<<(unsigned)t.first[t.n], WB_THREADS, lds, s>>>(t);
            }
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        for (int q = 0; q < t.n; ++q) {
            const WPBJob &j = jobs[idx[q]];
            const BwdScan &b = sc[idx[q]];
            const int64_t N = grid_size(j.g);
            {
                ProfScope prof_("gather_boxes", s);
                const bool last = j.V - v0 <= VCH;     // this scan's last chunk of views
                k_gather_boxes<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(
                    b.stage, j.g, b.lay.nb[0], b.lay.nb[1], b.lay.nb[2], last ? b.fix : nullptr,
                    b.vmax + j.V, j.g_ref);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
            {
                // the staged boxes are consumed: their buffer holds the range sums
                ProfScope prof_("coeff_reduce", s);
                const int vnc = vcs[q] * NC, nbk = b.lay.nbrick;
                const int64_t fit = (int64_t)nbk * HB3 / vnc;
                const int P = (int)std::max<int64_t>(1, std::min<int64_t>({256, nbk, fit}));
                const unsigned gx = (unsigned)((vnc + 255) / 256);
                k_reduce_coeff_parts<<<dim3(gx, (unsigned)P), 256, 0, s>>>(b.partial, nbk, vnc, P,
                                                                          b.stage);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                k_reduce_coeff_final<<<(unsigned)vnc, 256, 0, s>>>(b.stage, P, vnc,
                                                                   j.g_coeff + (int64_t)v0 * NC);
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    for (int k = 0; k < n; ++k) {
        const WPBJob &j = jobs[k];
        for (int l = 0; l < L; ++l) {
            if (!sc[k].staged[l]) continue;
            e = launch_upsample_adjoint(j.lv, l, j.lvl_grids[l], j.coeff, 1, j.g, nullptr,
                                        sc[k].staged[l], j.g_bases[l], sc[k].adjws, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t launch_warp_project_bwd(const float *ref, const GridK &g, const LevelsK &lv,
                                   const GridK *lvl_grids, const float *coeff, int V,
                                   const ConeK &c, const float *angles, const float *g_proj,
                                   float *g_ref, float *const *g_bases, float *g_coeff, void *ws,
                                   hipStream_t s) {
    WPBJob j;
    j.ref = ref;
    j.g = g;
    j.lv = lv;
    for (int l = 0; l < MAXL; ++l) {
        j.lvl_grids[l] = l < lv.L ? lvl_grids[l] : GridK{};
        j.g_bases[l] = l < lv.L ? g_bases[l] : nullptr;
    }
    j.coeff = coeff;
    j.V = V;
    j.c = c;
    j.angles = angles;
    j.g_proj = g_proj;
    j.g_ref = g_ref;
    j.g_coeff = g_coeff;
    j.ws = ws;
    return launch_warp_project_bwd_jobs(&j, 1, s);
}

}  // namespace pmf
