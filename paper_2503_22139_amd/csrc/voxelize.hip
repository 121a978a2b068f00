// voxelize.hip -- Eq. 5 (Gaussian voxelization) and its gradient.
//
// Forward: tile-binned splatting into LDS.  Each Gaussian's truncation
// ellipsoid is bounded by a box of voxels; Gaussians are binned into the
// tiles their box overlaps (count, scan, fill).  One workgroup owns a tile:
// its waves take the tile's Gaussians one at a time (parameters wave-uniform,
// held in scalar registers), evaluate them over box-and-tile column by column
// and add into an LDS copy of the tile in fixed point; the tile is then
// stored once with plain coalesced writes -- no global atomics.  Gaussians
// whose box spans more tiles than the bin capacity (e.g. untruncated ones) go
// to a separate list in ascending order, which every tile walks after its own
// list, adding in float per voxel in that order; neither sum depends on the
// order in which the binning's atomics filled the tile lists.
//
// Backward: Gaussian owner.  One wave per Gaussian walks the same voxel box,
// accumulates the per-Gaussian sums in registers and reduces them across the
// wave; lane 0 applies the chain rule through Sigma = R diag(s^2) R^T and the
// quaternion normalisation.
#include <math.h>

#include "pmf_internal.h"

namespace pmf {

struct alignas(16) GaussK {
    float mu[3];
    float a00;
    float a01, a02, a11, a12;
    float a22;
    int lo0, lo1, lo2;
    int hi0, hi1, hi2;
    int pad0, pad1;
};

struct GaussFull {
    float mu[3], s[3], qh[4], qn;
    float R[3][3];
    float A[3][3];
    int lo[3], hi[3];
};

// Sigma^-1 = R diag(s^-2) R^T and the voxel box that holds the ellipsoid
// m <= k^2 (half-extent k sqrt(Sigma_aa) per axis, widened by one voxel).
__device__ __forceinline__ void gauss_full(const float *__restrict__ mean,
                                           const float *__restrict__ scale,
                                           const float *__restrict__ quat, int64_t i, float k,
                                           const GridK &g, GaussFull &G) {
    for (int a = 0; a < 3; ++a) {
        G.mu[a] = mean[3 * i + a];
        G.s[a] = scale[3 * i + a];
    }
    float q[4];
    for (int c = 0; c < 4; ++c) q[c] = quat[4 * i + c];
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    G.qn = qn;
    for (int c = 0; c < 4; ++c) G.qh[c] = q[c] / qn;
    const float w = G.qh[0], x = G.qh[1], y = G.qh[2], z = G.qh[3];
    G.R[0][0] = 1.0f - 2.0f * (y * y + z * z);
    G.R[0][1] = 2.0f * (x * y - w * z);
    G.R[0][2] = 2.0f * (x * z + w * y);
    G.R[1][0] = 2.0f * (x * y + w * z);
    G.R[1][1] = 1.0f - 2.0f * (x * x + z * z);
    G.R[1][2] = 2.0f * (y * z - w * x);
    G.R[2][0] = 2.0f * (x * z - w * y);
    G.R[2][1] = 2.0f * (y * z + w * x);
    G.R[2][2] = 1.0f - 2.0f * (x * x + y * y);
    float is2[3], s2[3];
    for (int c = 0; c < 3; ++c) {
        s2[c] = G.s[c] * G.s[c];
        is2[c] = 1.0f / s2[c];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            G.A[a][b] = G.R[a][0] * G.R[b][0] * is2[0] + G.R[a][1] * G.R[b][1] * is2[1] +
                        G.R[a][2] * G.R[b][2] * is2[2];
    for (int a = 0; a < 3; ++a) {
        if (isinf(k)) {
            G.lo[a] = 0;
            G.hi[a] = g.n[a] - 1;
            continue;
        }
        const float var = G.R[a][0] * G.R[a][0] * s2[0] + G.R[a][1] * G.R[a][1] * s2[1] +
                          G.R[a][2] * G.R[a][2] * s2[2];
        const float ext = k * sqrtf(var);
        float l = floorf((G.mu[a] - ext - g.c0[a]) * g.inv_h[a]) - 1.0f;
        float u = ceilf((G.mu[a] + ext - g.c0[a]) * g.inv_h[a]) + 1.0f;
        l = fmaxf(l, 0.0f);
        u = fminf(u, (float)(g.n[a] - 1));
        if (!(l <= u)) {  // outside the grid (or NaN): empty box
            G.lo[a] = 1;
            G.hi[a] = 0;
        } else {
            G.lo[a] = (int)l;
            G.hi[a] = (int)u;
        }
    }
}

// Cheap test that Gaussian i's voxel box is empty without building it: the
// ellipsoid's half-extent on any axis is at most k max(s), and the box adds
// one voxel on each side (one more of margin here).  False when unsure
// (untruncated sets, NaN parameters), so callers then build the box.
__device__ __forceinline__ bool far_from_grid(const float *__restrict__ mean,
                                              const float *__restrict__ scale, int64_t i, float k,
                                              const GridK &g) {
    if (isinf(k)) return false;
    const float smax = fmaxf(fmaxf(fabsf(scale[3 * i]), fabsf(scale[3 * i + 1])),
                             fabsf(scale[3 * i + 2]));
    const float ext = 1.001f * k * smax;
    bool far = false;
    for (int a = 0; a < 3; ++a) {
        const float d = mean[3 * i + a] - g.c0[a];
        far = far || d + ext < -3.0f * g.h[a] || d - ext > (float)(g.n[a] + 2) * g.h[a];
    }
    return far;
}

__device__ __forceinline__ float quad(const GaussK &p, float d0, float d1, float d2) {
    const float t0 = fmaf(p.a00, d0, fmaf(p.a01, d1, p.a02 * d2));
    const float t1 = fmaf(p.a01, d0, fmaf(p.a11, d1, p.a12 * d2));
    const float t2 = fmaf(p.a02, d0, fmaf(p.a12, d1, p.a22 * d2));
    return fmaf(d0, t0, fmaf(d1, t1, d2 * t2));
}

// ---------------------------------------------------------------- binning
// Tile counters and cursors sit one per 128-byte line: the binning's atomics
// are device-scope and contend per line, and a packed array puts every
// tile's atomics on a few dozen lines.
constexpr int CNT_STRIDE = 32;

__global__ __launch_bounds__(256) void k_vox_prep(pmf_gauss_t gs, GridK g, float k, int T0,
                                                  int T1, int T2, int nt1, int nt2, int maxtiles,
                                                  GaussK *__restrict__ rec,
                                                  int32_t *__restrict__ tile_count,
                                                  int32_t *__restrict__ is_large) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= gs.m) return;
    is_large[i] = 0;
    if (far_from_grid(gs.mean, gs.scale, i, k, g)) {
        GaussK r = {};
        r.lo0 = r.lo1 = r.lo2 = 1;            // empty box: no tile, no voxel
        rec[i] = r;
        return;
    }
    GaussFull G;
    gauss_full(gs.mean, gs.scale, gs.quat, i, k, g, G);
    GaussK r;
    for (int a = 0; a < 3; ++a) r.mu[a] = G.mu[a];
    r.a00 = G.A[0][0];
    r.a01 = G.A[0][1];
    r.a02 = G.A[0][2];
    r.a11 = G.A[1][1];
    r.a12 = G.A[1][2];
    r.a22 = G.A[2][2];
    r.lo0 = G.lo[0];
    r.lo1 = G.lo[1];
    r.lo2 = G.lo[2];
    r.hi0 = G.hi[0];
    r.hi1 = G.hi[1];
    r.hi2 = G.hi[2];
    r.pad0 = r.pad1 = 0;
    rec[i] = r;
    if (G.lo[0] > G.hi[0] || G.lo[1] > G.hi[1] || G.lo[2] > G.hi[2]) return;
    const int t0a = G.lo[0] / T0, t0b = G.hi[0] / T0;
    const int t1a = G.lo[1] / T1, t1b = G.hi[1] / T1;
    const int t2a = G.lo[2] / T2, t2b = G.hi[2] / T2;
    const int64_t cnt = (int64_t)(t0b - t0a + 1) * (t1b - t1a + 1) * (t2b - t2a + 1);
    if (cnt > maxtiles) {
        is_large[i] = 1;
        return;
    }
    for (int a = t0a; a <= t0b; ++a)
        for (int b = t1a; b <= t1b; ++b)
            for (int c = t2a; c <= t2b; ++c)
                atomicAdd(&tile_count[((a * nt1 + b) * nt2 + c) * CNT_STRIDE], 1);
}

// Exclusive scan of n counts (CNT_STRIDE apart) by one workgroup of 1024
// threads: off[0..n] (dense), and the cursors (CNT_STRIDE apart) = off[] for
// the fill pass.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ cnt, int64_t n,
                                               int32_t *__restrict__ off,
                                               int32_t *__restrict__ cursor) {
    __shared__ int32_t part[1024];
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = threadIdx.x * per;
    const int64_t e = b + per < n ? b + per : n;
    int32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += cnt[i * CNT_STRIDE];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int32_t t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
    for (int64_t i = b; i < e; ++i) {
        off[i] = run;
        cursor[i * CNT_STRIDE] = run;
        run += cnt[i * CNT_STRIDE];
    }
    if (threadIdx.x == 1023) off[n] = part[1023];
}

// The large Gaussians in ascending index order (so that every tile adds
// them in one fixed order), by a three-step compaction: per block of 256
// Gaussians the count of large ones, an exclusive scan of the counts (one
// workgroup), and per block the positions of its large ones (ballots).
__global__ __launch_bounds__(256) void k_large_count(const int32_t *__restrict__ is_large,
                                                     int64_t m, int32_t *__restrict__ blk) {
    __shared__ int32_t part[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool f = i < m && is_large[i];
    const unsigned long long b = __ballot(f);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// In place: blk[0..n) counts -> exclusive offsets; *total = their sum.
__global__ __launch_bounds__(1024) void k_scan_counts(int32_t *__restrict__ blk, int n,
                                                      int32_t *__restrict__ total) {
    __shared__ int32_t part[1024];
    const int per = (n + 1023) / 1024;
    const int b = threadIdx.x * per;
    const int e = min(b + per, n);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += blk[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
    for (int i = b; i < e; ++i) {
        const int32_t c = blk[i];
        blk[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *total = part[1023];
}

__global__ __launch_bounds__(256) void k_large_fill(const int32_t *__restrict__ is_large,
                                                    int64_t m, const int32_t *__restrict__ blk,
                                                    int32_t *__restrict__ large) {
    __shared__ int32_t part[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool f = i < m && is_large[i];
    const unsigned long long b = __ballot(f);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) part[w] = __popcll(b);
    __syncthreads();
    int base = blk[blockIdx.x];
    for (int k = 0; k < w; ++k) base += part[k];
    const int below = __popcll(b & ((1ull << lane) - 1ull));
    if (f) large[base + below] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_vox_fill(int64_t m, const GaussK *__restrict__ rec,
                                                  int T0, int T1, int T2, int nt1, int nt2,
                                                  int maxtiles, int32_t *__restrict__ cursor,
                                                  int32_t *__restrict__ list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const GaussK r = rec[i];
    if (r.lo0 > r.hi0 || r.lo1 > r.hi1 || r.lo2 > r.hi2) return;
    const int t0a = r.lo0 / T0, t0b = r.hi0 / T0;
    const int t1a = r.lo1 / T1, t1b = r.hi1 / T1;
    const int t2a = r.lo2 / T2, t2b = r.hi2 / T2;
    const int64_t cnt = (int64_t)(t0b - t0a + 1) * (t1b - t1a + 1) * (t2b - t2a + 1);
    if (cnt > maxtiles) return;
    for (int a = t0a; a <= t0b; ++a)
        for (int b = t1a; b <= t1b; ++b)
            for (int c = t2a; c <= t2b; ++c)
                list[atomicAdd(&cursor[((a * nt1 + b) * nt2 + c) * CNT_STRIDE], 1)] = (int32_t)i;
}

// ------------------------------------------------------------ tile splat
// z range [za, zb] of column (ix, iy) that the truncation ellipsoid can
// reach: the roots of the quadratic in d2, widened by one voxel on each side
// and clipped to [lo2, hi2]; false when the column's quadratic stays clearly
// above k2.  Untruncated sets take the whole range.
__device__ __forceinline__ bool col_range(const GaussK &p, const GridK &g, float k2, bool untrunc,
                                          float d0, float d1, int lo2, int hi2, int &za,
                                          int &zb) {
    za = lo2;
    zb = hi2;
    if (untrunc) return true;
    // quad(d0, d1, d2) = a22 d2^2 + 2 bh d2 + cq
    const float bh = fmaf(p.a02, d0, p.a12 * d1);
    const float cq = fmaf(p.a00 * d0, d0, fmaf(2.0f * p.a01 * d0, d1, p.a11 * d1 * d1));
    float disc = fmaf(bh, bh, -p.a22 * (cq - k2));
    const float tol = 1e-4f * (fmaf(bh, bh, p.a22 * (fabsf(cq) + k2)));
    if (disc < -tol) return false;
    disc = fmaxf(disc, 0.0f);
    const float r = sqrtf(disc), inv_a = 1.0f / p.a22;
    // d2 range -> voxel index range: iz = (mu2 + d2 - c0_2) / h2
    const float inv_h2 = g.inv_h[2];
    const float zc = (p.mu[2] - g.c0[2]) * inv_h2;
    const float t_lo = zc + (-bh - r) * inv_a * inv_h2;
    const float t_hi = zc + (-bh + r) * inv_a * inv_h2;
    za = max(za, (int)floorf(t_lo) - 1);
    zb = min(zb, (int)ceilf(t_hi) + 1);
    return true;
}

// Evaluate a Gaussian over the voxel box [lo, hi] (inclusive) by (x, y)
// column: each lane takes a column and walks only its col_range, testing
// every voxel it visits with quad(); add(ix, iy, iz, e) for each in-mask
// voxel.
template <typename Add>
__device__ __forceinline__ void splat_cols(const GaussK &p, const GridK &g, float k2, int lo0,
                                           int lo1, int lo2, int hi0, int hi1, int hi2, Add add) {
    const int lane = threadIdx.x & 63;
    const int ny = hi1 - lo1 + 1;
    const int ncol = (hi0 - lo0 + 1) * ny;
    const bool untrunc = isinf(k2);
    for (int c0 = 0; c0 < ncol; c0 += 64) {
        const int col = c0 + lane;
        if (col >= ncol) continue;
        const int ix = lo0 + col / ny, iy = lo1 + col % ny;
        const float d0 = fmaf((float)ix, g.h[0], g.c0[0]) - p.mu[0];
        const float d1 = fmaf((float)iy, g.h[1], g.c0[1]) - p.mu[1];
        int za, zb;
        if (!col_range(p, g, k2, untrunc, d0, d1, lo2, hi2, za, zb)) continue;
        for (int iz = za; iz <= zb; ++iz) {
            const float d2 = fmaf((float)iz, g.h[2], g.c0[2]) - p.mu[2];
            const float mm = quad(p, d0, d1, d2);
            if (!(mm <= k2)) continue;
            add(ix, iy, iz, __expf(-0.5f * mm));
        }
    }
}

// One workgroup per tile.  Accumulation is in 32-bit fixed point with
// integer LDS atomics, so the sums do not depend on their order: per channel
// the scale is 2^30 / S with S = (Gaussians reaching the tile) x (their
// largest |value|), which bounds every voxel's sum since each Gaussian adds
// value * e (e <= 1) at most once per voxel, and is itself independent of
// the list's order.
constexpr int VT_CHUNK = 128;      // Gaussians staged in LDS at a time (one per thread)

// STAGE: the tile's Gaussians go through LDS VT_CHUNK at a time (one-channel
// sets, ~125 Gaussians per 8x16x16 tile); otherwise each wave reads its
// Gaussians directly (the many-channel MBC sets have ~16 per tile, where the
// barriers and the LDS cost more than they save).
template <bool STAGE>
__global__ __launch_bounds__(256) void k_vox_tile(const GaussK *__restrict__ rec,
                                                  const float *__restrict__ value, int C, GridK g,
                                                  float k2, int T0, int T1, int T2, int nt1,
                                                  int nt2, const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ large,
                                                  const int32_t *__restrict__ nlarge,
                                                  float *__restrict__ vol) {
    extern __shared__ int acc[];          // C tile planes, then VT_CHUNK x C staged values
    __shared__ float cs[4][16];
    __shared__ float scale[16];
    __shared__ GaussK gsh[STAGE ? VT_CHUNK : 1];
    const int tvox = T0 * T1 * T2;
    float *const vsh = (float *)(acc + C * tvox);
    for (int i = threadIdx.x; i < C * tvox; i += blockDim.x) acc[i] = 0;
    const int t = blockIdx.x;
    const int tz = t % nt2, ty = (t / nt2) % nt1, tx = t / (nt2 * nt1);
    const int b0 = tx * T0, b1 = ty * T1, b2 = tz * T2;
    const int e0 = min(b0 + T0, g.n[0]) - 1, e1 = min(b1 + T1, g.n[1]) - 1,
              e2 = min(b2 + T2, g.n[2]) - 1;
    const int beg = off[t], end = off[t + 1];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    const int nl = *nlarge;
    // per-channel bound S = (the tile's list length) x (the list's largest
    // |value|): every voxel's sum stays below it, and unlike a float sum of
    // the |values| it does not depend on the order the binning's atomics gave
    // the list, so neither does the scale (results repeat bit for bit)
    for (int c = 0; c < C; ++c) {
        float mx = 0.0f;
        for (int e = beg + (int)threadIdx.x; e < end; e += blockDim.x)
            mx = fmaxf(mx, fabsf(value[(int64_t)list[e] * C + c]));
        mx = wave_max(mx);
        if (lane == 0) cs[wave][c] = mx;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)C) {
        const float mx = fmaxf(fmaxf(cs[0][threadIdx.x], cs[1][threadIdx.x]),
                               fmaxf(cs[2][threadIdx.x], cs[3][threadIdx.x]));
        const float S = (float)(end - beg) * mx;
        scale[threadIdx.x] = S > 0.0f ? 1073741824.0f / (S * 1.0001f) : 0.0f;
    }
    // Staged: each thread fetches one record and its values, so a wave does
    // not wait for two dependent global reads per Gaussian; the integer sums
    // do not depend on the order.
    if constexpr (!STAGE) {
        __syncthreads();
        for (int e = beg + wave; e < end; e += nw) {
            const int gi = __builtin_amdgcn_readfirstlane(list[e]);
            const GaussK p = rec[gi];
            const int lo0 = max(p.lo0, b0), lo1 = max(p.lo1, b1), lo2 = max(p.lo2, b2);
            const int hi0 = min(p.hi0, e0), hi1 = min(p.hi1, e1), hi2 = min(p.hi2, e2);
            if (lo0 > hi0 || lo1 > hi1 || lo2 > hi2) continue;
            const float *vv = value + (int64_t)gi * C;
            splat_cols(p, g, k2, lo0, lo1, lo2, hi0, hi1, hi2, [&](int ix, int iy, int iz, float ev) {
                const int li = ((ix - b0) * T1 + (iy - b1)) * T2 + (iz - b2);
                for (int c = 0; c < C; ++c)
                    atomicAdd(&acc[c * tvox + li], __float2int_rn(vv[c] * scale[c] * ev));
            });
        }
    }
    for (int cb = beg; STAGE && cb < end; cb += VT_CHUNK) {
        const int n = min(VT_CHUNK, end - cb);
        __syncthreads();
        if ((int)threadIdx.x < n) {
            const int gi = list[cb + threadIdx.x];
            gsh[threadIdx.x] = rec[gi];
            for (int c = 0; c < C; ++c) vsh[threadIdx.x * C + c] = value[(int64_t)gi * C + c];
        }
        __syncthreads();
        for (int e = wave; e < n; e += nw) {
            GaussK p = gsh[e];
            const int lo0 = max(p.lo0, b0), lo1 = max(p.lo1, b1), lo2 = max(p.lo2, b2);
            const int hi0 = min(p.hi0, e0), hi1 = min(p.hi1, e1), hi2 = min(p.hi2, e2);
            if (lo0 > hi0 || lo1 > hi1 || lo2 > hi2) continue;
            const float *vv = vsh + e * C;
            splat_cols(p, g, k2, lo0, lo1, lo2, hi0, hi1, hi2, [&](int ix, int iy, int iz, float ev) {
                const int li = ((ix - b0) * T1 + (iy - b1)) * T2 + (iz - b2);
                for (int c = 0; c < C; ++c)
                    atomicAdd(&acc[c * tvox + li], __float2int_rn(vv[c] * scale[c] * ev));
            });
        }
    }
    __syncthreads();
    // fixed point -> float, in place
    float *const accf = (float *)acc;
    for (int i = threadIdx.x; i < C * tvox; i += blockDim.x) {
        const float sc = scale[i / tvox];
        accf[i] = sc > 0.0f ? (float)acc[i] / sc : 0.0f;
    }
    // Gaussians too large for the bins (e.g. untruncated sets): each thread
    // owns voxels of the tile and adds them in float, in the list's ascending
    // order (a fixed order: the results repeat bit for bit)
    if (nl > 0) {
        __syncthreads();
        for (int li = threadIdx.x; li < tvox; li += blockDim.x) {
            const int ix = b0 + li / (T1 * T2), iy = b1 + (li / T2) % T1, iz = b2 + li % T2;
            if (ix > e0 || iy > e1 || iz > e2) continue;
            const float d0g = fmaf((float)ix, g.h[0], g.c0[0]);
            const float d1g = fmaf((float)iy, g.h[1], g.c0[1]);
            const float d2g = fmaf((float)iz, g.h[2], g.c0[2]);
            for (int e = 0; e < nl; ++e) {
                const int gi = __builtin_amdgcn_readfirstlane(large[e]);
                const GaussK p = rec[gi];
                if (ix < p.lo0 || ix > p.hi0 || iy < p.lo1 || iy > p.hi1 || iz < p.lo2 ||
                    iz > p.hi2)
                    continue;
                const float mm = quad(p, d0g - p.mu[0], d1g - p.mu[1], d2g - p.mu[2]);
                if (!(mm <= k2)) continue;
                const float ev = __expf(-0.5f * mm);
                const float *vv = value + (int64_t)gi * C;
                for (int c = 0; c < C; ++c) accf[c * tvox + li] += vv[c] * ev;
            }
        }
    }
    __syncthreads();
    const int64_t N = grid_size(g);
    for (int i = threadIdx.x; i < C * tvox; i += blockDim.x) {
        const int c = i / tvox, li = i % tvox;
        const int z = li % T2, y = (li / T2) % T1, x = li / (T2 * T1);
        const int gx = b0 + x, gy = b1 + y, gz = b2 + z;
        if (gx < g.n[0] && gy < g.n[1] && gz < g.n[2])
            vol[(int64_t)c * N + ((int64_t)gx * g.n[1] + gy) * g.n[2] + gz] = accf[i];
    }
}

VoxPlan vox_plan(int64_t m, int c, const GridK &g) {
    VoxPlan p;
    int T[3];
    if (c <= 1) {
        T[0] = 8; T[1] = 16; T[2] = 16;     // 16^3 measured slower (denser tiles)
    } else if (c <= 4) {
        T[0] = 8; T[1] = 16; T[2] = 16;
    } else if (c <= 9) {
        T[0] = 8; T[1] = 8; T[2] = 16;
    } else {
        T[0] = 8; T[1] = 8; T[2] = 8;
    }
    // small grids (a TV sub-volume): halve the longest tile edge, down to 8,
    // until there are at least 256 tiles to spread over the CUs
    auto ntiles_of = [&](const int *t) {
        int64_t n = 1;
        for (int a = 0; a < 3; ++a) n *= (g.n[a] + t[a] - 1) / t[a];
        return n;
    };
    while (ntiles_of(T) < 256) {
        int a = 0;
        for (int b = 1; b < 3; ++b)
            if (T[b] > T[a]) a = b;
        if (T[a] <= 8) break;
        T[a] /= 2;
    }
    p.ntiles = 1;
    for (int a = 0; a < 3; ++a) {
        p.T[a] = T[a];
        p.nt[a] = (g.n[a] + T[a] - 1) / T[a];
        p.ntiles *= p.nt[a];
    }
    p.maxtiles = 32;
    p.cap = m * p.maxtiles;
    return p;
}

size_t vox_workspace(const VoxPlan &p, int64_t m) {
    size_t s = 0;
    s += align256(sizeof(GaussK) * (size_t)(m > 0 ? m : 1));  // records
    s += align256(sizeof(int32_t) * CNT_STRIDE * (size_t)p.ntiles);   // counts
    s += align256(sizeof(int32_t) * (size_t)(p.ntiles + 1));          // offsets
    s += align256(sizeof(int32_t) * CNT_STRIDE * (size_t)p.ntiles);   // cursors
    s += align256(sizeof(int32_t) * (size_t)(p.cap > 0 ? p.cap : 1));  // list
    s += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));  // large list
    s += align256(sizeof(int32_t));                            // large count
    s += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));  // large flags
    s += align256(sizeof(int32_t) * (size_t)((m + 255) / 256 + 1));   // per-block counts
    return s;
}

hipError_t launch_voxelize(const pmf_gauss_t &gs, const GridK &g, float k, float *vol,
                           const VoxPlan &p, void *ws, hipStream_t s) {
    char *w = (char *)ws;
    const int64_t m = gs.m;
    GaussK *rec = (GaussK *)w;
    w += align256(sizeof(GaussK) * (size_t)(m > 0 ? m : 1));
    int32_t *cnt = (int32_t *)w;
    w += align256(sizeof(int32_t) * CNT_STRIDE * (size_t)p.ntiles);
    int32_t *off = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)(p.ntiles + 1));
    int32_t *cur = (int32_t *)w;
    w += align256(sizeof(int32_t) * CNT_STRIDE * (size_t)p.ntiles);
    int32_t *list = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)(p.cap > 0 ? p.cap : 1));
    int32_t *large = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *nlarge = (int32_t *)w;
    w += align256(sizeof(int32_t));
    int32_t *is_large = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *blk = (int32_t *)w;

    const float k2 = isinf(k) ? INFINITY : k * k;
    hipError_t e = launch_fill_i32(cnt, CNT_STRIDE * p.ntiles, 0, s);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(nlarge, 1, 0, s);
    if (e != hipSuccess) return e;
    if (m > 0) {
        {
            ProfScope prof_("voxelize_prep", s);
            k_vox_prep<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(
                gs, g, k, p.T[0], p.T[1], p.T[2], p.nt[1], p.nt[2], p.maxtiles, rec, cnt, is_large);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int nblk = (int)((m + 255) / 256);
        k_large_count<<<(unsigned)nblk, 256, 0, s>>>(is_large, m, blk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_scan_counts<<<1, 1024, 0, s>>>(blk, nblk, nlarge);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_large_fill<<<(unsigned)nblk, 256, 0, s>>>(is_large, m, blk, large);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        ProfScope prof_("voxelize_scan", s);
        k_scan<<<1, 1024, 0, s>>>(cnt, p.ntiles, off, cur);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (m > 0) {
        {
            ProfScope prof_("voxelize_fill", s);
            k_vox_fill<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, rec, p.T[0], p.T[1], p.T[2],
                                                                  p.nt[1], p.nt[2], p.maxtiles, cur,
                                                                  list);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const bool stage = gs.c == 1;
    const size_t lds =
        sizeof(float) * (size_t)gs.c * (p.T[0] * p.T[1] * p.T[2] + (stage ? VT_CHUNK : 0));
    {
        ProfScope prof_("voxelize_tile", s);
        if (stage)
            k_vox_tile<true><<<(unsigned)p.ntiles, 256, lds, s>>>(
                rec, gs.value, gs.c, g, k2, p.T[0], p.T[1], p.T[2], p.nt[1], p.nt[2], off, list,
                large, nlarge, vol);
        else
            k_vox_tile<false><<<(unsigned)p.ntiles, 256, lds, s>>>(
                rec, gs.value, gs.c, g, k2, p.T[0], p.T[1], p.T[2], p.nt[1], p.nt[2], off, list,
                large, nlarge, vol);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- backward
constexpr int MAXC = 16;

// CT > 0: the channel count at compile time (the loads of a voxel's channels
// issue together); CT = 0: any C up to MAXC.
template <int CT>
__global__ __launch_bounds__(256) void k_vox_bwd(pmf_gauss_t gs, GridK g, float k,
                                                 const float *__restrict__ g_vol,
                                                 pmf_gauss_grad_t gr) {
    const int64_t gi = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (gi >= gs.m) return;
    const int lane = threadIdx.x & 63;
    const int C = CT > 0 ? CT : gs.c;
    if (far_from_grid(gs.mean, gs.scale, gi, k, g)) {     // wave-uniform: no voxel, zero gradients
        if (lane == 63) {
            for (int c = 0; c < C; ++c) gr.value[gi * C + c] = 0.0f;
            for (int a = 0; a < 3; ++a) {
                gr.mean[3 * gi + a] = 0.0f;
                gr.scale[3 * gi + a] = 0.0f;
            }
            for (int c = 0; c < 4; ++c) gr.quat[4 * gi + c] = 0.0f;
        }
        return;
    }
    GaussFull G;
    gauss_full(gs.mean, gs.scale, gs.quat, gi, k, g, G);
    GaussK p;
    for (int a = 0; a < 3; ++a) p.mu[a] = G.mu[a];
    p.a00 = G.A[0][0];
    p.a01 = G.A[0][1];
    p.a02 = G.A[0][2];
    p.a11 = G.A[1][1];
    p.a12 = G.A[1][2];
    p.a22 = G.A[2][2];
    const float k2 = isinf(k) ? INFINITY : k * k;
    const float *vv = gs.value + gi * C;
    float val[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) val[c] = c < C ? vv[c] : 0.0f;
    float gv[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) gv[c] = 0.0f;
    float gm0 = 0, gm1 = 0, gm2 = 0;
    float M00 = 0, M01 = 0, M02 = 0, M11 = 0, M12 = 0, M22 = 0;
    const int64_t N = grid_size(g);
    // Column walk of splat_cols with the same voxels in the same order per
    // lane; every voxel of the column range is loaded (the range lies in the
    // grid) and voxels outside the ellipsoid add exact zeros, so the loop has
    // no branch and the loads of successive voxels overlap.
    if (G.lo[0] <= G.hi[0] && G.lo[1] <= G.hi[1] && G.lo[2] <= G.hi[2]) {
        const int ny = G.hi[1] - G.lo[1] + 1;
        const int ncol = (G.hi[0] - G.lo[0] + 1) * ny;
        const bool untrunc = isinf(k2);
        for (int c0 = 0; c0 < ncol; c0 += 64) {
            const int col = c0 + lane;
            if (col >= ncol) continue;
            const int ix = G.lo[0] + col / ny, iy = G.lo[1] + col % ny;
            const float d0 = fmaf((float)ix, g.h[0], g.c0[0]) - p.mu[0];
            const float d1 = fmaf((float)iy, g.h[1], g.c0[1]) - p.mu[1];
            int za, zb;
            if (!col_range(p, g, k2, untrunc, d0, d1, G.lo[2], G.hi[2], za, zb)) continue;
            const float *gcol = g_vol + ((int64_t)ix * g.n[1] + iy) * g.n[2];
            constexpr int UNR = CT == 1 ? 4 : 2;     // voxels whose loads overlap
#pragma unroll UNR
            for (int iz = za; iz <= zb; ++iz) {
                float gl[MAXC];
#pragma unroll
                for (int c = 0; c < MAXC; ++c)
                    if (c < C) gl[c] = gcol[c * N + iz];
                const float d2 = fmaf((float)iz, g.h[2], g.c0[2]) - p.mu[2];
                const float mm = quad(p, d0, d1, d2);
                const bool in = mm <= k2;
                const float ev = in ? __expf(-0.5f * mm) : 0.0f;
                float Gj = 0.0f;
#pragma unroll
                for (int c = 0; c < MAXC; ++c) {
                    if (c < C) {
                        const float gc = in ? gl[c] : 0.0f;
                        gv[c] = fmaf(gc, ev, gv[c]);
                        Gj = fmaf(val[c], gc, Gj);
                    }
                }
                const float t = Gj * ev;
                const float A0 = fmaf(p.a00, d0, fmaf(p.a01, d1, p.a02 * d2));
                const float A1 = fmaf(p.a01, d0, fmaf(p.a11, d1, p.a12 * d2));
                const float A2 = fmaf(p.a02, d0, fmaf(p.a12, d1, p.a22 * d2));
                gm0 = fmaf(t, A0, gm0);
                gm1 = fmaf(t, A1, gm1);
                gm2 = fmaf(t, A2, gm2);
                const float ht = -0.5f * t;
                M00 = fmaf(ht * d0, d0, M00);
                M01 = fmaf(ht * d0, d1, M01);
                M02 = fmaf(ht * d0, d2, M02);
                M11 = fmaf(ht * d1, d1, M11);
                M12 = fmaf(ht * d1, d2, M12);
                M22 = fmaf(ht * d2, d2, M22);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
        if (c < C) gv[c] = wave_sum_lane63(gv[c]);
    gm0 = wave_sum_lane63(gm0);
    gm1 = wave_sum_lane63(gm1);
    gm2 = wave_sum_lane63(gm2);
    M00 = wave_sum_lane63(M00);
    M01 = wave_sum_lane63(M01);
    M02 = wave_sum_lane63(M02);
    M11 = wave_sum_lane63(M11);
    M12 = wave_sum_lane63(M12);
    M22 = wave_sum_lane63(M22);
    if (lane != 63) return;
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
        if (c < C) gr.value[gi * C + c] = gv[c];
    gr.mean[3 * gi + 0] = gm0;
    gr.mean[3 * gi + 1] = gm1;
    gr.mean[3 * gi + 2] = gm2;
    const float M[3][3] = {{M00, M01, M02}, {M01, M11, M12}, {M02, M12, M22}};
    float MR[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            MR[a][b] = M[a][0] * G.R[0][b] + M[a][1] * G.R[1][b] + M[a][2] * G.R[2][b];
    for (int kk = 0; kk < 3; ++kk) {
        const float d = G.R[0][kk] * MR[0][kk] + G.R[1][kk] * MR[1][kk] + G.R[2][kk] * MR[2][kk];
        gr.scale[3 * gi + kk] = -2.0f * d / (G.s[kk] * G.s[kk] * G.s[kk]);
    }
    float GR[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) GR[a][b] = 2.0f * MR[a][b] / (G.s[b] * G.s[b]);
    const float w = G.qh[0], x = G.qh[1], y = G.qh[2], z = G.qh[3];
    float gq[4];
    gq[0] = 2.0f * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] +
                    x * GR[2][1]);
    gq[1] = 2.0f * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - 2.0f * x * GR[1][1] -
                    w * GR[1][2] + z * GR[2][0] + w * GR[2][1] - 2.0f * x * GR[2][2]);
    gq[2] = 2.0f * (-2.0f * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] +
                    z * GR[1][2] - w * GR[2][0] + z * GR[2][1] - 2.0f * y * GR[2][2]);
    gq[3] = 2.0f * (-2.0f * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] -
                    2.0f * z * GR[1][1] + y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
    const float dot = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
    for (int c = 0; c < 4; ++c) gr.quat[4 * gi + c] = (gq[c] - G.qh[c] * dot) / G.qn;
}

hipError_t launch_voxelize_bwd(const pmf_gauss_t &gs, const GridK &g, float k, const float *g_vol,
                               const pmf_gauss_grad_t &gr, hipStream_t s) {
    if (gs.m <= 0) return hipSuccess;
    {
        ProfScope prof_("voxelize_bwd", s);
        const unsigned nb = (unsigned)((gs.m + 3) / 4);
        if (gs.c == 1)
            k_vox_bwd<1><<<nb, 256, 0, s>>>(gs, g, k, g_vol, gr);
        else if (gs.c == 3)
            k_vox_bwd<3><<<nb, 256, 0, s>>>(gs, g, k, g_vol, gr);
        else if (gs.c == 9)
            k_vox_bwd<9><<<nb, 256, 0, s>>>(gs, g, k, g_vol, gr);
        else
            k_vox_bwd<0><<<nb, 256, 0, s>>>(gs, g, k, g_vol, gr);
    }
    return hipGetLastError();
}

}  // namespace pmf
