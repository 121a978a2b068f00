// combine.hip -- the low-rank DVF of Eq. 3 and its adjoint.
//
// Forward: one thread per output voxel.  For each level the trilinear
// stencil on the level grid is computed once and shared by its 3B channels;
// the L*B*3 sampled basis values stay in registers while the V views'
// displacements are formed from the (wave-uniform) coefficients.
//
// Adjoint, coefficients: the same per-voxel basis samples dotted with g_dvf,
// reduced per workgroup into a partial buffer and summed in a second pass
// (fixed order, deterministic).
//
// Adjoint, bases: the trilinear upsampling is a tensor product of three 1-D
// interpolation matrices (fine index -> level index per axis, zero rows
// outside the box), so its transpose is applied as up to three 1-D gather
// passes, each recomputing the forward's 1-D weights.  Axes on which the
// level grid equals the output grid are skipped.
#include <math.h>

#include "pmf_internal.h"

namespace pmf {

template <int L, int B>
__global__ __launch_bounds__(256) void k_combine(LevelsK lv, const float *__restrict__ coeff,
                                                 int V, GridK out, float *__restrict__ dvf) {
    const int64_t N = grid_size(out);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int iz = (int)(j % out.n[2]);
    const int iy = (int)((j / out.n[2]) % out.n[1]);
    const int ix = (int)(j / ((int64_t)out.n[2] * out.n[1]));
    float sv[L][B][3];
    basis_samples<L, B>(lv, ix, iy, iz, sv);
    for (int v = 0; v < V; ++v) {
        const float *cv = coeff + (int64_t)v * L * B * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float d = 0.0f;
#pragma unroll
            for (int l = 0; l < L; ++l)
#pragma unroll
                for (int b = 0; b < B; ++b) d = fmaf(cv[(l * B + b) * 3 + k], sv[l][b][k], d);
            dvf[((int64_t)v * 3 + k) * N + j] = d;
        }
    }
}

hipError_t launch_combine(const LevelsK &lv, const float *coeff, int V, const GridK &out, float *dvf,
                          hipStream_t s) {
    const int64_t N = grid_size(out);
    return dispatch_lb(lv.L, lv.B, [&](auto Lc, auto Bc) {
        constexpr int L = decltype(Lc)::value, B = decltype(Bc)::value;
        {
            ProfScope prof_("combine", s);
            k_combine<L, B><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(lv, coeff, V, out, dvf);
        }
        return hipGetLastError();
    });
}

// ------------------------------------------------------- coefficient adjoint
constexpr int NLB = MAXL * MAXB * 3;
constexpr int CB_BLOCKS = 1024;

template <int L, int B>
__global__ __launch_bounds__(256) void k_combine_bwd_coeff(LevelsK lv, GridK out,
                                                           const float *__restrict__ g_dvf,
                                                           float *__restrict__ partial) {
    const int64_t N = grid_size(out);
    const int v = blockIdx.y;
    float acc[L][B][3];
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[l][b][k] = 0.0f;
    const float *gd = g_dvf + (int64_t)v * 3 * N;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int iz = (int)(j % out.n[2]);
        const int iy = (int)((j / out.n[2]) % out.n[1]);
        const int ix = (int)(j / ((int64_t)out.n[2] * out.n[1]));
        float sv[L][B][3];
        basis_samples<L, B>(lv, ix, iy, iz, sv);
        const float g[3] = {gd[j], gd[N + j], gd[2 * N + j]};
#pragma unroll
        for (int l = 0; l < L; ++l)
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int k = 0; k < 3; ++k) acc[l][b][k] = fmaf(g[k], sv[l][b][k], acc[l][b][k]);
    }
    __shared__ float red[4][NLB];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float t = wave_sum_lane63(acc[l][b][k]);
                if (lane == 63) red[wave][(l * B + b) * 3 + k] = t;
            }
    __syncthreads();
    if (threadIdx.x < L * B * 3) {
        const int idx = threadIdx.x;
        const float t = (red[0][idx] + red[1][idx]) + (red[2][idx] + red[3][idx]);
        partial[((int64_t)v * gridDim.x + blockIdx.x) * NLB + idx] = t;
    }
}

// g_coeff[v][l][b][k] = sum over blocks of the partials: one workgroup per
// output entry, fixed-order tree (deterministic).
__global__ __launch_bounds__(256) void k_reduce_coeff(const float *__restrict__ partial, int nblk,
                                                      int per, float *__restrict__ g_coeff) {
    const int t = blockIdx.x;
    const int v = t / per, idx = t % per;
    float s = 0.0f;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x)
        s += partial[((int64_t)v * nblk + i) * NLB + idx];
    __shared__ float red[4];
    s = wave_sum_lane63(s);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) g_coeff[t] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ----------------------------------------------------------- basis adjoint
// Source of the first pass: channel c of level l is
//   sum_v coeff[v][l][b][k] g_dvf[v][k][j]   (c = b*3 + k), or G[c][j].
struct AdjSrc {
    const float *g_dvf;
    const float *coeff;
    const float *G;
    int V, L, B, l;
    int64_t N;
};

__device__ __forceinline__ float adj_src(const AdjSrc &src, int c, int64_t j) {
    if (src.G) return src.G[(int64_t)c * src.N + j];
    const int b = c / 3, k = c % 3;
    float s = 0.0f;
    for (int v = 0; v < src.V; ++v)
        s = fmaf(src.coeff[(((int64_t)v * src.L + src.l) * src.B + b) * 3 + k],
                 src.g_dvf[((int64_t)v * 3 + k) * src.N + j], s);
    return s;
}

struct Shape4 {
    int c, d[3];
};

// One 1-D transpose pass along axis `ax`, out[c][..p..] = sum_j W(j,p)
// in[c][..j..] with W(j,p) the forward's linear weight of level index p for
// fine index j.  Each line along `ax` is cut into nseg segments of outputs
// [p0, p1), one thread each (short or few lines would otherwise leave the
// pass latency-bound): the thread walks the line's input values from the
// first one that reaches p0, in order, each split between its two level
// cells (weights 1 - f and f, as the forward reads them), and emits its
// outputs in order (a cell is complete once the walk has passed it).  Every
// output sums its terms in ascending fine order whatever nseg is.
__global__ __launch_bounds__(256) void k_adj_line(Shape4 in_s, int ax, int nc, float scale,
                                                  float off, int nseg,
                                                  const float *__restrict__ in, AdjSrc src,
                                                  float *__restrict__ out) {
    // lines: all index tuples of (c, d0, d1, d2) with the ax index fixed to 0
    int ld[3] = {in_s.d[0], in_s.d[1], in_s.d[2]};
    ld[ax] = 1;
    const int64_t nlines = (int64_t)in_s.c * ld[0] * ld[1] * ld[2];
    const int64_t tt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tt >= nlines * nseg) return;
    // segment-major, so neighbouring threads take neighbouring lines
    const int seg = (int)(tt / nlines);
    int64_t r = tt - (int64_t)seg * nlines;
    const int per = (nc + nseg - 1) / nseg;
    const int p0 = seg * per, p1 = min(nc, p0 + per);
    if (p0 >= p1) return;
    int idx[3];
    idx[2] = (int)(r % ld[2]);
    r /= ld[2];
    idx[1] = (int)(r % ld[1]);
    r /= ld[1];
    idx[0] = (int)(r % ld[0]);
    const int c = (int)(r / ld[0]);
    const int nf = in_s.d[ax];
    // input strides and base (channel-major [c][d0][d1][d2])
    const int64_t ist = ax == 2 ? 1 : (ax == 1 ? in_s.d[2] : (int64_t)in_s.d[1] * in_s.d[2]);
    const int64_t ibase = ((int64_t)idx[0] * in_s.d[1] + idx[1]) * in_s.d[2] + idx[2];
    const int64_t cbase = (int64_t)c * in_s.d[0] * in_s.d[1] * in_s.d[2];
    // output shape: ax dimension nc
    int od[3] = {in_s.d[0], in_s.d[1], in_s.d[2]};
    od[ax] = nc;
    const int64_t ost = ax == 2 ? 1 : (ax == 1 ? od[2] : (int64_t)od[1] * od[2]);
    const int64_t obase = (((int64_t)c * od[0] + idx[0]) * od[1] + idx[1]) * od[2] + idx[2];
    auto emit = [&](int p, float v) {
        if (p >= p0 && p < p1) out[obase + (int64_t)p * ost] = v;
    };
    // a value at cell i feeds outputs i and i + 1: start a little below the
    // first fine index whose cell is p0 - 1 (values below it are skipped)
    const int jlo = p0 == 0 ? 0 : max(0, (int)floorf(((float)(p0 - 1) - off) / scale) - 2);
    int next = p0;          // first output not yet written
    int cur = -1;           // cell of the pending pair (cur, cur + 1)
    float a0 = 0.0f, a1 = 0.0f;
    bool done = false;
    // The line's values are fetched ADJ_U at a time ahead of the walk (whose
    // branches would otherwise leave one load in flight per wave).
    constexpr int ADJ_U = 8;
    for (int j0 = jlo; j0 < nf && !done; j0 += ADJ_U) {
        float xs[ADJ_U];
#pragma unroll
        for (int u = 0; u < ADJ_U; ++u) {
            const int64_t jj = min(j0 + u, nf - 1);     // past the end: in range, unused
            xs[u] = in ? in[cbase + ibase + jj * ist] : adj_src(src, c, ibase + jj * ist);
        }
#pragma unroll
        for (int u = 0; u < ADJ_U; ++u) {
            const int j = j0 + u;
            if (j >= nf) break;
            int i;
            float f;
            if (!axis_cell(fmaf((float)j, scale, off), nc, i, f)) continue;
            if (i < p0 - 1) continue;           // reaches no output of this segment
            if (i >= p1) {                      // nor does anything past it
                done = true;
                break;
            }
            if (i != cur) {
                // cells below i are complete: write them (zeros for cells no value reached)
                if (cur >= 0) {
                    emit(cur, a0);
                    next = cur + 1;
                    a0 = (cur + 1 == i) ? a1 : 0.0f;
                    if (cur + 1 < i) {
                        emit(cur + 1, a1);
                        next = cur + 2;
                    }
                } else {
                    a0 = 0.0f;
                }
                for (; next < i; ++next) emit(next, 0.0f);
                a1 = 0.0f;
                cur = i;
            }
            const float x = xs[u];
            a0 = fmaf(1.0f - f, x, a0);
            a1 = fmaf(f, x, a1);
        }
    }
    if (cur >= 0) {
        emit(cur, a0);
        emit(cur + 1, a1);
        next = max(next, cur + 2);
    }
    for (; next < p1; ++next) emit(next, 0.0f);
}

// Level grid equals the output grid: the source is the answer.
__global__ __launch_bounds__(256) void k_adj_copy(int C, int64_t N, AdjSrc src,
                                                  float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)C * N) return;
    out[t] = adj_src(src, (int)(t / N), t % N);
}

static void adj_plan(const GridK &out, const AxisMap &m, int C, int order[3], int &np,
                     size_t &bufA, size_t &bufB) {
    np = 0;
    for (int a = 0; a < 3; ++a)
        if (!m.ident[a]) order[np++] = a;
    int d[3] = {out.n[0], out.n[1], out.n[2]};
    size_t sz[3] = {0, 0, 0};
    for (int p = 0; p < np; ++p) {
        d[order[p]] = m.n[order[p]];
        sz[p] = (size_t)C * d[0] * d[1] * d[2];
    }
    bufA = np >= 2 ? sz[0] : 0;
    bufB = np >= 3 ? sz[1] : 0;
}

size_t upsample_adjoint_workspace(int C, const GridK &lvl_grid, const GridK &out, const AxisMap &m) {
    (void)lvl_grid;
    int order[3], np;
    size_t a, b;
    adj_plan(out, m, C, order, np, a, b);
    return align256(a * sizeof(float)) + align256(b * sizeof(float));
}

hipError_t launch_upsample_adjoint(const LevelsK &lv, int l, const GridK &lvl_grid,
                                   const float *coeff, int V, const GridK &out, const float *g_dvf,
                                   const float *G, float *g_base, void *ws, hipStream_t s) {
    (void)lvl_grid;
    const AxisMap &m = lv.map[l];
    const int C = 3 * lv.B;
    AdjSrc src;
    src.g_dvf = g_dvf;
    src.coeff = coeff;
    src.G = G;
    src.V = V;
    src.L = lv.L;
    src.B = lv.B;
    src.l = l;
    src.N = grid_size(out);
    int order[3], np;
    size_t a, b;
    adj_plan(out, m, C, order, np, a, b);
    if (np == 0) {
        const int64_t tot = (int64_t)C * src.N;
        {
            ProfScope prof_("upsample_adjoint", s);
            k_adj_copy<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(C, src.N, src, g_base);
        }
        return hipGetLastError();
    }
    float *bufA = (float *)ws;
    float *bufB = (float *)((char *)ws + align256(a * sizeof(float)));
    Shape4 sh;
    sh.c = C;
    sh.d[0] = out.n[0];
    sh.d[1] = out.n[1];
    sh.d[2] = out.n[2];
    const float *in = nullptr;
    for (int p = 0; p < np; ++p) {
        const int ax = order[p];
        float *dst = (p == np - 1) ? g_base : (p == 0 ? bufA : bufB);
        Shape4 os = sh;
        os.d[ax] = m.n[ax];
        const int64_t lines = (int64_t)sh.c * sh.d[0] * sh.d[1] * sh.d[2] / sh.d[ax];
        // segments per line: enough threads to cover the pass's latency
        // (about 2^20: measured against 2^18 to 2^22), at least 8 outputs each
        int nseg = 1;
        while (2 * nseg <= m.n[ax] / 8 && lines * nseg < (1 << 20)) nseg *= 2;
        const int64_t threads = lines * nseg;
        {
            ProfScope prof_("upsample_adjoint", s);
            k_adj_line<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(
                sh, ax, m.n[ax], m.scale[ax], m.off[ax], nseg, in, src, dst);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        in = dst;
        sh = os;
    }
    return hipSuccess;
}

size_t combine_bwd_workspace(const LevelsK &lv, const GridK *lvl_grids, int V, const GridK &out) {
    size_t part = align256(sizeof(float) * (size_t)CB_BLOCKS * (size_t)V * NLB);
    size_t adj = 0;
    for (int l = 0; l < lv.L; ++l) {
        size_t w = upsample_adjoint_workspace(3 * lv.B, lvl_grids[l], out, lv.map[l]);
        if (w > adj) adj = w;
    }
    return part + adj;
}

hipError_t launch_combine_bwd(const LevelsK &lv, const GridK *lvl_grids, const float *coeff, int V,
                              const GridK &out, const float *g_dvf, float *const *g_bases,
                              float *g_coeff, void *ws, hipStream_t s) {
    const int64_t N = grid_size(out);
    int nblk = (int)((N + 255) / 256);
    if (nblk > CB_BLOCKS) nblk = CB_BLOCKS;
    float *partial = (float *)ws;
    char *adjws = (char *)ws + align256(sizeof(float) * (size_t)CB_BLOCKS * (size_t)V * NLB);
    hipError_t e = dispatch_lb(lv.L, lv.B, [&](auto Lc, auto Bc) {
        constexpr int L = decltype(Lc)::value, B = decltype(Bc)::value;
        {
            ProfScope prof_("combine_bwd_coeff", s);
            k_combine_bwd_coeff<L, B>
                <<<dim3((unsigned)nblk, (unsigned)V), 256, 0, s>>>(lv, out, g_dvf, partial);
        }
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    const int per = lv.L * lv.B * 3;
    const int tot = V * per;
    {
        ProfScope prof_("combine_bwd_reduce", s);
        k_reduce_coeff<<<(unsigned)tot, 256, 0, s>>>(partial, nblk, per, g_coeff);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int l = 0; l < lv.L; ++l) {
        e = launch_upsample_adjoint(lv, l, lvl_grids[l], coeff, V, out, g_dvf, nullptr, g_bases[l],
                                    adjws, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pmf
