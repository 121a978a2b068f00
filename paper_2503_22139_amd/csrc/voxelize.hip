// voxelize.hip -- Eq. 5 (Gaussian voxelization) and its gradient.
//
// Forward: tile-binned.  Each Gaussian's truncation ellipsoid is bounded by
// a box of voxels; Gaussians are binned into the tiles their box overlaps
// (count, scan, fill).  One workgroup owns a tile.  One-channel sets (the
// reference, ~150 Gaussians per tile) are splatted: the waves lay the
// (Gaussian, column) pairs of batches of the tile's Gaussians over their
// lanes and add into an LDS copy of the tile in fixed point.  Three- and
// nine-channel sets (the MBC bases, ~10 Gaussians per tile) are gathered:
// each thread owns a few voxels and keeps their channel sums in registers.
// Either way the tile is stored once with plain writes -- no global atomics
// -- and the integer sums do not depend on the order in which the binning's
// atomics filled the tile lists.  Gaussians whose box spans more tiles than
// the bin capacity (e.g. untruncated ones) go to a separate list in
// ascending order, which every tile walks after its own list, adding in
// float per voxel in that order.
//
// Backward: Gaussian owner.  A wave takes a batch of Gaussians, walks each
// one's voxel box, accumulates the per-Gaussian sums in registers and
// reduces them across the wave; one lane per Gaussian applies the chain rule
// through Sigma = R diag(s^2) R^T and the quaternion normalisation.
#include <math.h>

#include "pmf_internal.h"

namespace pmf {

constexpr int MAXC_VOX = 16;     // channels per Gaussian set (voxelize_workspace checks)

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

// ---------------------------------------------------------------- binning
// Tile counters sit one per 128-byte line: the count pass's atomics are
// device-scope and contend per line, and a packed array puts every tile's
// atomics on a few dozen lines.  Each atomic's old value is the pair's place
// in its tile's list, so the fill pass writes the lists without atomics.
constexpr int CNT_STRIDE = 32;

__global__ __launch_bounds__(256) void k_vox_prep(pmf_gauss_t gs, GridK g, float k, int T0,
                                                  int T1, int T2, int nt1, int nt2, int maxtiles,
                                                  GaussK *__restrict__ rec,
                                                  int32_t *__restrict__ tile_count,
                                                  int32_t *__restrict__ slot,
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
    // the count's old value is this pair's place in the tile's list: kept
    // (pair q of Gaussian i at slot[q m + i]) so the fill needs no atomics
    int q = 0;
    for (int a = t0a; a <= t0b; ++a)
        for (int b = t1a; b <= t1b; ++b)
            for (int c = t2a; c <= t2b; ++c, ++q)
                slot[(int64_t)q * gs.m + i] =
                    atomicAdd(&tile_count[((a * nt1 + b) * nt2 + c) * CNT_STRIDE], 1);
}

// Exclusive scan of n counts (CNT_STRIDE apart) by one workgroup of 1024
// threads: off[0..n] (dense).  Each thread takes a run of up to SCAN_U counts (loaded
// together and kept in registers for the second pass); the block's scan is
// a DPP scan per wave plus the wave totals.
constexpr int SCAN_U = 8;
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ cnt, int64_t n,
                                               int32_t *__restrict__ off) {
    __shared__ int32_t wsum[16];
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = threadIdx.x * per;
    const int64_t e = b + per < n ? b + per : n;
    const bool few = per <= SCAN_U;       // uniform
    int32_t v[SCAN_U];
    int32_t s = 0;
    if (few) {
#pragma unroll
        for (int k = 0; k < SCAN_U; ++k) v[k] = b + k < e ? cnt[(b + k) * CNT_STRIDE] : 0;
#pragma unroll
        for (int k = 0; k < SCAN_U; ++k) s += v[k];
    } else {
        for (int64_t i = b; i < e; ++i) s += cnt[i * CNT_STRIDE];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t incl = wave_incl_sum(s);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int32_t base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    int32_t run = base + incl - s;
    if (few) {
#pragma unroll
        for (int k = 0; k < SCAN_U; ++k) {
            if (b + k < e) {
                off[b + k] = run;
                run += v[k];
            }
        }
    } else {
        for (int64_t i = b; i < e; ++i) {
            off[i] = run;
            run += cnt[i * CNT_STRIDE];
        }
    }
    if (threadIdx.x == 1023) off[n] = base + incl;
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
                                                  int maxtiles, const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ slot,
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
    // the pairs in the count pass's order, each to the place that pass drew
    int q = 0;
    for (int a = t0a; a <= t0b; ++a)
        for (int b = t1a; b <= t1b; ++b)
            for (int c = t2a; c <= t2b; ++c, ++q)
                list[off[(a * nt1 + b) * nt2 + c] + slot[(int64_t)q * m + i]] = (int32_t)i;
}

// ------------------------------------------------------------ tile splat
// On a column (d0, d1 fixed) the quadratic form is m(d2) = a22 d2^2 + b2 d2
// + cq; the forward and the adjoint evaluate it in this form, so both take
// the same mask decisions.
__device__ __forceinline__ void col_coeffs(float a00, float a01, float a02, float a11, float a12,
                                           float d0, float d1, float &b2, float &cq) {
    b2 = 2.0f * fmaf(a02, d0, a12 * d1);
    cq = fmaf(a00 * d0, d0, fmaf(2.0f * a01 * d0, d1, a11 * d1 * d1));
}

__device__ __forceinline__ float col_quad(float a22, float b2, float cq, float d2) {
    return fmaf(fmaf(a22, d2, b2), d2, cq);
}

// z range [za, zb] of a column that the truncation ellipsoid m <= k2 can
// reach: the roots of m(d2) = k2, widened by one voxel on each side and
// clipped to [lo2, hi2]; false when the column's quadratic stays clearly
// above k2.  Untruncated sets take the whole range.
__device__ __forceinline__ bool col_range(float a22, float b2, float cq, float zc, float inv_h2,
                                          float k2, bool untrunc, int lo2, int hi2, int &za,
                                          int &zb) {
    za = lo2;
    zb = hi2;
    if (untrunc) return true;
    const float bh = 0.5f * b2;
    float disc = fmaf(bh, bh, -a22 * (cq - k2));
    const float tol = 1e-4f * (fmaf(bh, bh, a22 * (fabsf(cq) + k2)));
    if (disc < -tol) return false;
    disc = fmaxf(disc, 0.0f);
    const float r = sqrtf(disc), inv_a = 1.0f / a22;
    // d2 range -> voxel index range: iz = zc + d2 / h2, zc = (mu2 - c0_2) / h2
    const float t_lo = zc + (-bh - r) * inv_a * inv_h2;
    const float t_hi = zc + (-bh + r) * inv_a * inv_h2;
    za = max(za, (int)floorf(t_lo) - 1);
    zb = min(zb, (int)ceilf(t_hi) + 1);
    return true;
}

// One workgroup per tile.  Accumulation is in 32-bit fixed point with
// integer LDS atomics, so the sums do not depend on their order: per channel
// the scale is 2^30 / S with S = (Gaussians reaching the tile) x (their
// largest |value|), which bounds every voxel's sum since each Gaussian adds
// value * e (e <= 1) at most once per voxel, and is itself independent of
// the list's order.
//
// Work layout: each wave takes batches of up to VB of the tile's Gaussians
// (lane j < VB reads batch entry j, clips its box to the tile and stages it
// in LDS), then lays the batch's (Gaussian, column) pairs out over its
// lanes, 64 at a time: a lane finds its pair by a search over the batch's
// column offsets, walks the column's z range (col_range: nearly every voxel
// it visits is inside the ellipsoid) and adds value x e^(-m/2) of each
// in-mask voxel.  The lanes are spread over the columns of many Gaussians,
// not one Gaussian's few.
constexpr int VB = 16;

struct VoxB {                 // one Gaussian of a wave's batch, box clipped to the tile
    float mu[3];
    float a00, a01, a02, a11, a12, a22;
    int lo0, lo1, lo2, hi2, ny, cend;    // its columns are [cend - ncols, cend)
    int ncols;
};

template <int T0, int T1, int T2, int CT>
__global__ __launch_bounds__(256) void k_vox_tile(const GaussK *__restrict__ rec,
                                                  const float *__restrict__ value, int Crt, GridK g,
                                                  float k2, int nt1, int nt2,
                                                  const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ large,
                                                  const int32_t *__restrict__ nlarge,
                                                  float *__restrict__ vol) {
    constexpr int TV = T0 * T1 * T2;
    constexpr int NW = 4;
    constexpr int CM = CT > 0 ? CT : MAXC_VOX;
    const int C = CT > 0 ? CT : Crt;
    extern __shared__ int acc[];          // C tile planes
    __shared__ float cs[NW][CM];
    __shared__ float scale[CM];
    __shared__ VoxB bt[NW][VB];
    __shared__ float bv[NW][VB][CM];      // value x scale per batch entry
    for (int i = threadIdx.x; i < C * TV; i += 256) acc[i] = 0;
    const int t = blockIdx.x;
    const int tz = t % nt2, ty = (t / nt2) % nt1, tx = t / (nt2 * nt1);
    const int b0 = tx * T0, b1 = ty * T1, b2 = tz * T2;
    const int e0 = min(b0 + T0, g.n[0]) - 1, e1 = min(b1 + T1, g.n[1]) - 1,
              e2 = min(b2 + T2, g.n[2]) - 1;
    const int beg = off[t], end = off[t + 1];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nl = *nlarge;
    // per-channel bound S = (the tile's list length) x (the list's largest
    // |value|): every voxel's sum stays below it, and unlike a float sum of
    // the |values| it does not depend on the order the binning's atomics gave
    // the list, so neither does the scale (results repeat bit for bit)
    for (int c = 0; c < C; ++c) {
        float mx = 0.0f;
        for (int e = beg + (int)threadIdx.x; e < end; e += 256)
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
    __syncthreads();
    const bool untrunc = isinf(k2);
    const float inv_h2 = g.inv_h[2];
    VoxB *const B = bt[wave];
    for (int eb = beg + wave * VB; eb < end; eb += NW * VB) {     // uniform per wave
        const int nb = min(VB, end - eb);
        int ncols = 0;
        VoxB q;
        if (lane < nb) {
            const int gi = list[eb + lane];
            const GaussK p = rec[gi];
            const int lo0 = max(p.lo0, b0), lo1 = max(p.lo1, b1), lo2 = max(p.lo2, b2);
            const int hi0 = min(p.hi0, e0), hi1 = min(p.hi1, e1), hi2 = min(p.hi2, e2);
            if (lo0 <= hi0 && lo1 <= hi1 && lo2 <= hi2) ncols = (hi0 - lo0 + 1) * (hi1 - lo1 + 1);
            for (int a = 0; a < 3; ++a) q.mu[a] = p.mu[a];
            q.a00 = p.a00;
            q.a01 = p.a01;
            q.a02 = p.a02;
            q.a11 = p.a11;
            q.a12 = p.a12;
            q.a22 = p.a22;
            q.lo0 = lo0;
            q.lo1 = lo1;
            q.lo2 = lo2;
            q.hi2 = hi2;
            q.ny = hi1 - lo1 + 1;
            q.ncols = ncols;
            const float *vv = value + (int64_t)gi * C;
            for (int c = 0; c < C; ++c) bv[wave][lane][c] = vv[c] * scale[c];
        }
        const int cend = wave_incl_sum(ncols);          // lanes >= nb add 0
        const int total = __builtin_amdgcn_readlane(cend, VB - 1);
        if (lane < nb) {
            q.cend = cend;
            B[lane] = q;
        } else if (lane < VB) {          // the search reads every entry's cend
            B[lane].cend = cend;
            B[lane].ncols = 0;
        }
        wave_lds_sync();
        for (int cb = 0; cb < total; cb += 64) {           // uniform per wave
            const int qc = cb + lane;
            if (qc >= total) continue;
            // batch entry: the smallest j with cend_j > qc
            int j = 0;
#pragma unroll
            for (int step = VB / 2; step > 0; step >>= 1)
                if (B[j + step - 1].cend <= qc) j += step;
            const VoxB &q = B[j];
            const int ql = qc - (q.cend - q.ncols);
            // column ql of the clipped box, y fastest (exact: ql < 256, ny <= 16)
            const int cx = (int)(((float)ql + 0.5f) * __builtin_amdgcn_rcpf((float)q.ny));
            const int ix = q.lo0 + cx, iy = q.lo1 + (ql - cx * q.ny);
            const float d0 = fmaf((float)ix, g.h[0], g.c0[0]) - q.mu[0];
            const float d1 = fmaf((float)iy, g.h[1], g.c0[1]) - q.mu[1];
            float cb2, cq;
            col_coeffs(q.a00, q.a01, q.a02, q.a11, q.a12, d0, d1, cb2, cq);
            int za, zb;
            if (!col_range(q.a22, cb2, cq, (q.mu[2] - g.c0[2]) * inv_h2, inv_h2, k2, untrunc,
                           q.lo2, q.hi2, za, zb))
                continue;
            const float a22 = q.a22, mu2 = q.mu[2];
            float vs[CM];
#pragma unroll
            for (int c = 0; c < CM; ++c) vs[c] = c < C ? bv[wave][j][c] : 0.0f;
            int li = ((ix - b0) * T1 + (iy - b1)) * T2 + (za - b2);
            for (int iz = za; iz <= zb; ++iz, ++li) {
                const float d2 = fmaf((float)iz, g.h[2], g.c0[2]) - mu2;
                const float mm = col_quad(a22, cb2, cq, d2);
                if (!(mm <= k2)) continue;
                const float ev = __expf(-0.5f * mm);
#pragma unroll
                for (int c = 0; c < CM; ++c)
                    if (c < C) atomicAdd(&acc[c * TV + li], __float2int_rn(vs[c] * ev));
            }
        }
        wave_lds_sync();
    }
    __syncthreads();
    // fixed point -> float, in place
    float *const accf = (float *)acc;
    for (int i = threadIdx.x; i < C * TV; i += 256) {
        const float sc = scale[i / TV];
        accf[i] = sc > 0.0f ? (float)acc[i] / sc : 0.0f;
    }
    // Gaussians too large for the bins (e.g. untruncated sets): each thread
    // owns voxels of the tile and adds them in float, in the list's ascending
    // order (a fixed order: the results repeat bit for bit)
    if (nl > 0) {
        __syncthreads();
        for (int li = threadIdx.x; li < TV; li += 256) {
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
                float cb2, cq;
                col_coeffs(p.a00, p.a01, p.a02, p.a11, p.a12, d0g - p.mu[0], d1g - p.mu[1], cb2, cq);
                const float mm = col_quad(p.a22, cb2, cq, d2g - p.mu[2]);
                if (!(mm <= k2)) continue;
                const float ev = __expf(-0.5f * mm);
                const float *vv = value + (int64_t)gi * C;
                for (int c = 0; c < C; ++c) accf[c * TV + li] += vv[c] * ev;
            }
        }
    }
    __syncthreads();
    const int64_t N = grid_size(g);
    for (int i = threadIdx.x; i < C * TV; i += 256) {
        const int c = i / TV, li = i % TV;
        const int z = li % T2, y = (li / T2) % T1, x = li / (T2 * T1);
        const int gx = b0 + x, gy = b1 + y, gz = b2 + z;
        if (gx < g.n[0] && gy < g.n[1] && gz < g.n[2])
            vol[(int64_t)c * N + ((int64_t)gx * g.n[1] + gy) * g.n[2] + gz] = accf[i];
    }
}

// Multi-channel sets (the MBC bases: few Gaussians per tile, 3 or 9
// channels): voxel owners.  A thread owns SEG consecutive voxels of one
// column of the tile and keeps their channel sums in registers, in the same
// 32-bit fixed point and with the same per-term rounding as k_vox_tile (so
// the two give the same bits, and the sums do not depend on the order of the
// tile's list); the tile's Gaussians are staged in LDS a chunk at a time and
// every thread tests each against its voxels.  No LDS accumulator, no
// atomics: the kernel holds little LDS and keeps many tiles in flight.
constexpr int VG_CHUNK = 64;

template <int T0, int T1, int T2, int CT>
__global__ __launch_bounds__(256) void k_vox_gather(const GaussK *__restrict__ rec,
                                                    const float *__restrict__ value, GridK g,
                                                    float k2, int nt1, int nt2,
                                                    const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ large,
                                                    const int32_t *__restrict__ nlarge,
                                                    float *__restrict__ vol) {
    constexpr int TV = T0 * T1 * T2;
    constexpr int SEG = TV / 256;           // voxels per thread (along z)
    constexpr int NS = T2 / SEG;            // threads per column
    static_assert(SEG >= 1 && T2 % SEG == 0 && TV % 256 == 0, "tile shape");
    __shared__ GaussK gsh[VG_CHUNK];
    __shared__ float gvs[VG_CHUNK][CT];
    __shared__ float cs[4][CT];
    __shared__ float scale[CT];
    const int t = blockIdx.x;
    const int tz = t % nt2, ty = (t / nt2) % nt1, tx = t / (nt2 * nt1);
    const int b0 = tx * T0, b1 = ty * T1, b2 = tz * T2;
    const int e0 = min(b0 + T0, g.n[0]) - 1, e1 = min(b1 + T1, g.n[1]) - 1,
              e2 = min(b2 + T2, g.n[2]) - 1;
    const int beg = off[t], end = off[t + 1];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int seg = threadIdx.x % NS, col = threadIdx.x / NS;
    const int ix = b0 + col / T1, iy = b1 + col % T1, z0 = b2 + seg * SEG;
    // x range of the wave's columns (a wave-uniform cull of each Gaussian)
    const int wx0 = b0 + (wave * 64 / NS) / T1, wx1 = b0 + ((wave * 64 + 63) / NS) / T1;
    {
        // one pass over the list: each entry's channels load together
        float mx[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) mx[c] = 0.0f;
        for (int e = beg + (int)threadIdx.x; e < end; e += 256) {
            const float *vv = value + (int64_t)list[e] * CT;
#pragma unroll
            for (int c = 0; c < CT; ++c) mx[c] = fmaxf(mx[c], fabsf(vv[c]));
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const float m = wave_max(mx[c]);
            if (lane == 0) cs[wave][c] = m;
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)CT) {
        const float mx = fmaxf(fmaxf(cs[0][threadIdx.x], cs[1][threadIdx.x]),
                               fmaxf(cs[2][threadIdx.x], cs[3][threadIdx.x]));
        const float S = (float)(end - beg) * mx;
        scale[threadIdx.x] = S > 0.0f ? 1073741824.0f / (S * 1.0001f) : 0.0f;
    }
    const float d0g = fmaf((float)ix, g.h[0], g.c0[0]);
    const float d1g = fmaf((float)iy, g.h[1], g.c0[1]);
    float d2g[SEG];
#pragma unroll
    for (int s = 0; s < SEG; ++s) d2g[s] = fmaf((float)(z0 + s), g.h[2], g.c0[2]);
    int acc[SEG][CT];
#pragma unroll
    for (int s = 0; s < SEG; ++s)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[s][c] = 0;
    for (int cb = beg; cb < end; cb += VG_CHUNK) {
        const int n = min(VG_CHUNK, end - cb);
        __syncthreads();                  // scale ready / previous chunk consumed
        if ((int)threadIdx.x < n) {
            const int gi = list[cb + threadIdx.x];
            gsh[threadIdx.x] = rec[gi];
            for (int c = 0; c < CT; ++c) gvs[threadIdx.x][c] = value[(int64_t)gi * CT + c] * scale[c];
        }
        __syncthreads();
        for (int e = 0; e < n; ++e) {
            const GaussK p = gsh[e];
            if (p.hi0 < wx0 || p.lo0 > wx1 || p.hi1 < b1 || p.lo1 > e1 || p.hi2 < b2 || p.lo2 > e2)
                continue;                                     // uniform
            if (ix < p.lo0 || ix > p.hi0 || iy < p.lo1 || iy > p.hi1 || z0 > p.hi2 ||
                z0 + SEG - 1 < p.lo2)
                continue;
            float cb2, cq;
            col_coeffs(p.a00, p.a01, p.a02, p.a11, p.a12, d0g - p.mu[0], d1g - p.mu[1], cb2, cq);
#pragma unroll
            for (int s = 0; s < SEG; ++s) {
                const float mm = col_quad(p.a22, cb2, cq, d2g[s] - p.mu[2]);
                if (z0 + s >= p.lo2 && z0 + s <= p.hi2 && mm <= k2) {
                    const float ev = __expf(-0.5f * mm);
#pragma unroll
                    for (int c = 0; c < CT; ++c) acc[s][c] += __float2int_rn(gvs[e][c] * ev);
                }
            }
        }
    }
    float out[SEG][CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const float sc = scale[c];
#pragma unroll
        for (int s = 0; s < SEG; ++s) out[s][c] = sc > 0.0f ? (float)acc[s][c] / sc : 0.0f;
    }
    // Gaussians too large for the bins, in float, in the list's ascending
    // order (as k_vox_tile)
    const int nl = *nlarge;
    for (int e = 0; e < nl; ++e) {
        const int gi = __builtin_amdgcn_readfirstlane(large[e]);
        const GaussK p = rec[gi];
        if (ix < p.lo0 || ix > p.hi0 || iy < p.lo1 || iy > p.hi1) continue;
        float cb2, cq;
        col_coeffs(p.a00, p.a01, p.a02, p.a11, p.a12, d0g - p.mu[0], d1g - p.mu[1], cb2, cq);
#pragma unroll
        for (int s = 0; s < SEG; ++s) {
            if (z0 + s < p.lo2 || z0 + s > p.hi2) continue;
            const float mm = col_quad(p.a22, cb2, cq, d2g[s] - p.mu[2]);
            if (!(mm <= k2)) continue;
            const float ev = __expf(-0.5f * mm);
#pragma unroll
            for (int c = 0; c < CT; ++c) out[s][c] += value[(int64_t)gi * CT + c] * ev;
        }
    }
    if (ix > e0 || iy > e1) return;
    const int64_t N = grid_size(g);
    float *const vb = vol + ((int64_t)ix * g.n[1] + iy) * g.n[2];
    if constexpr (SEG == 4) {
        // a thread's four voxels as one 16-byte store per channel when the
        // rows and the volume are 16-byte aligned (z0 is a multiple of 4)
        if ((g.n[2] & 3) == 0 && ((uintptr_t)vol & 15) == 0 && z0 + 3 <= e2) {
#pragma unroll
            for (int c = 0; c < CT; ++c)
                *(float4 *)(vb + (int64_t)c * N + z0) =
                    make_float4(out[0][c], out[1][c], out[2][c], out[3][c]);
            return;
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int s = 0; s < SEG; ++s)
            if (z0 + s <= e2) vb[(int64_t)c * N + z0 + s] = out[s][c];
}

VoxPlan vox_plan(int64_t m, int c, const GridK &g) {
    VoxPlan p;
    int T[3];
    if (c <= 1) {
        // 200k Gaussians into 256x256x128, binning + tiles: 8x16x16 0.50 ms
        // (tiles 0.307), 8x8x32 0.49 ms (tiles 0.275: fewer columns cut at
        // z faces, a little more binning), 8x16x32 0.66 ms and 8x8x64
        // 0.63 ms (fewer, longer lists: the per-tile atomics contend)
        T[0] = 8; T[1] = 8; T[2] = 32;
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
    s += align256(sizeof(int32_t) * (size_t)(p.cap > 0 ? p.cap : 1));  // list
    s += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));  // large list
    s += align256(sizeof(int32_t));                            // large count
    s += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));  // large flags
    s += align256(sizeof(int32_t) * (size_t)((m + 255) / 256 + 1));   // per-block counts
    s += align256(sizeof(int32_t) * (size_t)(p.cap > 0 ? p.cap : 1));  // list places
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
    int32_t *list = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)(p.cap > 0 ? p.cap : 1));
    int32_t *large = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *nlarge = (int32_t *)w;
    w += align256(sizeof(int32_t));
    int32_t *is_large = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *blk = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)((m + 255) / 256 + 1));
    int32_t *slot = (int32_t *)w;

    const float k2 = isinf(k) ? INFINITY : k * k;
    hipError_t e = launch_fill_i32(cnt, CNT_STRIDE * p.ntiles, 0, s);
    if (e != hipSuccess) return e;
    // with Gaussians, k_scan_counts writes the large-list length
    if (m == 0 && (e = launch_fill_i32(nlarge, 1, 0, s)) != hipSuccess) return e;
    if (m > 0) {
        {
            ProfScope prof_("voxelize_prep", s);
            k_vox_prep<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(
                gs, g, k, p.T[0], p.T[1], p.T[2], p.nt[1], p.nt[2], p.maxtiles, rec, cnt, slot,
                is_large);
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
        k_scan<<<1, 1024, 0, s>>>(cnt, p.ntiles, off);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (m > 0) {
        {
            ProfScope prof_("voxelize_fill", s);
            k_vox_fill<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, rec, p.T[0], p.T[1], p.T[2],
                                                                  p.nt[1], p.nt[2], p.maxtiles, off,
                                                                  slot, list);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const size_t lds = sizeof(float) * (size_t)gs.c * (p.T[0] * p.T[1] * p.T[2]);
    {
        ProfScope prof_("voxelize_tile", s);
        const int sel = (p.T[1] == 16 ? 2 : 0) + (p.T[2] == 16 ? 1 : 0);
        const int cs = gs.c;
        // one channel: the LDS splat (many Gaussians per tile); 3 or 9
        // channels: voxel owners; other channel counts: the LDS splat
#define VOX_TILE(T1_, T2_, CT_)                                                                   \
    k_vox_tile<8, T1_, T2_, CT_><<<(unsigned)p.ntiles, 256, lds, s>>>(                           \
        rec, gs.value, gs.c, g, k2, p.nt[1], p.nt[2], off, list, large, nlarge, vol)
#define VOX_GATHER(T1_, T2_, CT_)                                                                 \
    k_vox_gather<8, T1_, T2_, CT_><<<(unsigned)p.ntiles, 256, 0, s>>>(                           \
        rec, gs.value, g, k2, p.nt[1], p.nt[2], off, list, large, nlarge, vol)
#define VOX_TILE_C(T1_, T2_)                                                                      \
    do {                                                                                          \
        if (cs == 1) VOX_TILE(T1_, T2_, 1);                                                       \
        else if (cs == 3) VOX_GATHER(T1_, T2_, 3);                                                \
        else if (cs == 9) VOX_GATHER(T1_, T2_, 9);                                                \
        else VOX_TILE(T1_, T2_, 0);                                                               \
    } while (0)
        if (cs == 1 && p.T[1] == 8 && p.T[2] == 32) VOX_TILE(8, 32, 1);   // one channel
        else switch (sel) {
            case 3: VOX_TILE_C(16, 16); break;
            case 2: VOX_TILE_C(16, 8); break;
            case 1: VOX_TILE_C(8, 16); break;
            default: VOX_TILE_C(8, 8); break;
        }
#undef VOX_TILE_C
#undef VOX_GATHER
#undef VOX_TILE
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- backward

// Adjoint, Gaussian owner.  A wave takes `per` consecutive Gaussians; lane
// j < per builds Gaussian j's geometry and stages what the walk needs in
// LDS.  The wave then walks each Gaussian's voxel box in turn with the
// forward's columns (64 columns at a time over the lanes, z along each
// lane's col_range) and accumulates per lane, with t = e sum_c v_c g_c:
//   sum e g_c (value gradients),
//   sum t d    (mean gradient A sum t d),
//   sum t d d^T (the gradient of the quadratic form),
// where on a column (d0, d1 fixed) only sum t, sum t d2 and sum t d2^2 are
// kept per voxel and folded into the others when the lane leaves the
// column.  The sums are reduced across the wave, and at the end lane j
// applies the chain rule through Sigma^-1 = R diag(s^-2) R^T and the
// quaternion normalisation to Gaussian j.
constexpr int BW_NS = 9;       // sums besides the channels: P0..P2, M00 M01 M02 M11 M12 M22

struct VoxG {                  // one Gaussian of the wave's batch
    float mu[3];
    float a00, a01, a02, a11, a12, a22;
    int lo0, lo1, lo2, hi0, hi1, hi2;
};

//
// ZL: the multi-channel layout.  Each voxel then loads C values, and lanes on
// different columns would touch a cache line per lane per channel; instead
// the lanes of a wave sit along z (zl lanes per column, 64 / zl columns per
// step) so each load covers a few lines, and every voxel accumulates its
// terms directly.
template <int CT, bool ZL>
__global__ __launch_bounds__(64) void k_vox_bwd(pmf_gauss_t gs, GridK g, float k, int per,
                                                const float *__restrict__ g_vol,
                                                pmf_gauss_grad_t gr) {
    constexpr int CM = CT > 0 ? CT : MAXC_VOX;
    const int C = CT > 0 ? CT : gs.c;
    // LDS for the wave's `per` Gaussians only (a one-Gaussian batch leaves
    // room for many waves per CU): records, values, reduced sums
    extern __shared__ float4 bwd_smem[];
    VoxG *const gb = (VoxG *)bwd_smem;
    float(*const gval)[CM] = (float(*)[CM])(gb + per);
    float(*const sums)[CM + BW_NS] = (float(*)[CM + BW_NS])(gval + per);
    const int lane = threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * per;
    const float k2 = isinf(k) ? INFINITY : k * k;
    const bool untrunc = isinf(k2);
    // set-up: lane j < per builds Gaussian g0 + j
    if (lane < per) {
        const int64_t gi = g0 + lane;
        VoxG q = {};
        q.lo0 = q.lo1 = q.lo2 = 1;                  // empty box
        if (gi < gs.m && !far_from_grid(gs.mean, gs.scale, gi, k, g)) {
            GaussFull G;
            gauss_full(gs.mean, gs.scale, gs.quat, gi, k, g, G);
            for (int a = 0; a < 3; ++a) q.mu[a] = G.mu[a];
            q.a00 = G.A[0][0];
            q.a01 = G.A[0][1];
            q.a02 = G.A[0][2];
            q.a11 = G.A[1][1];
            q.a12 = G.A[1][2];
            q.a22 = G.A[2][2];
            q.lo0 = G.lo[0];
            q.lo1 = G.lo[1];
            q.lo2 = G.lo[2];
            q.hi0 = G.hi[0];
            q.hi1 = G.hi[1];
            q.hi2 = G.hi[2];
            for (int c = 0; c < C; ++c) gval[lane][c] = gs.value[gi * C + c];
        }
        gb[lane] = q;
    }
    __syncthreads();
    const int64_t N = grid_size(g);
    const float inv_h2 = g.inv_h[2];
    const int nj = (int)min((int64_t)per, gs.m - g0);
    for (int j = 0; j < nj; ++j) {                  // uniform
        const VoxG q = gb[j];
        float gv[CM];
#pragma unroll
        for (int c = 0; c < CM; ++c) gv[c] = 0.0f;
        float P0 = 0, P1 = 0, P2 = 0, M00 = 0, M01 = 0, M02 = 0, M11 = 0, M12 = 0, M22 = 0;
        if (q.lo0 <= q.hi0 && q.lo1 <= q.hi1 && q.lo2 <= q.hi2) {
            float val[CM];
#pragma unroll
            for (int c = 0; c < CM; ++c) val[c] = c < C ? gval[j][c] : 0.0f;
            const int ny = q.hi1 - q.lo1 + 1;
            const int ncol = (q.hi0 - q.lo0 + 1) * ny;
            const float rny = __builtin_amdgcn_rcpf((float)ny);
            const float zc = (q.mu[2] - g.c0[2]) * inv_h2;
            if constexpr (ZL) {
                const int nz = q.hi2 - q.lo2 + 1;
                const int zl = nz <= 4 ? 4 : nz <= 8 ? 8 : nz <= 16 ? 16 : nz <= 32 ? 32 : 64;
                const int cpr = 64 / zl;
                const int zr = lane & (zl - 1), cl = lane / zl;
                for (int c0 = 0; c0 < ncol; c0 += cpr) {
                    const int col = c0 + cl;
                    if (col >= ncol) continue;
                    int cx = (int)(((float)col + 0.5f) * rny);
                    int cy = col - cx * ny;
                    if (cy < 0) {
                        --cx;
                        cy += ny;
                    } else if (cy >= ny) {
                        ++cx;
                        cy -= ny;
                    }
                    const int ix = q.lo0 + cx, iy = q.lo1 + cy;
                    const float d0 = fmaf((float)ix, g.h[0], g.c0[0]) - q.mu[0];
                    const float d1 = fmaf((float)iy, g.h[1], g.c0[1]) - q.mu[1];
                    float cb2, cq;
                    col_coeffs(q.a00, q.a01, q.a02, q.a11, q.a12, d0, d1, cb2, cq);
                    int za, zb;
                    if (!col_range(q.a22, cb2, cq, zc, inv_h2, k2, untrunc, q.lo2, q.hi2, za, zb))
                        continue;
                    const float *gcol = g_vol + ((int64_t)ix * g.n[1] + iy) * g.n[2];
                    for (int iz = za + zr; iz <= zb; iz += zl) {
                        float gl[CM];
#pragma unroll
                        for (int c = 0; c < CM; ++c)
                            if (c < C) gl[c] = gcol[c * N + iz];
                        const float d2 = fmaf((float)iz, g.h[2], g.c0[2]) - q.mu[2];
                        const float mm = col_quad(q.a22, cb2, cq, d2);
                        const float ev = mm <= k2 ? __expf(-0.5f * mm) : 0.0f;
                        float Gj = 0.0f;
#pragma unroll
                        for (int c = 0; c < CM; ++c) {
                            if (c < C) {
                                gv[c] = fmaf(gl[c], ev, gv[c]);
                                Gj = fmaf(val[c], gl[c], Gj);
                            }
                        }
                        const float t = Gj * ev;
                        const float t0 = t * d0, t1 = t * d1, t2 = t * d2;
                        P0 += t0;
                        P1 += t1;
                        P2 += t2;
                        M00 = fmaf(t0, d0, M00);
                        M01 = fmaf(t0, d1, M01);
                        M02 = fmaf(t0, d2, M02);
                        M11 = fmaf(t1, d1, M11);
                        M12 = fmaf(t1, d2, M12);
                        M22 = fmaf(t2, d2, M22);
                    }
                }
            } else
            for (int c0 = 0; c0 < ncol; c0 += 64) {
                const int col = c0 + lane;
                if (col >= ncol) continue;
                // col = cx * ny + cy (the float quotient is corrected to exact)
                int cx = (int)(((float)col + 0.5f) * rny);
                int cy = col - cx * ny;
                if (cy < 0) {
                    --cx;
                    cy += ny;
                } else if (cy >= ny) {
                    ++cx;
                    cy -= ny;
                }
                const int ix = q.lo0 + cx, iy = q.lo1 + cy;
                const float d0 = fmaf((float)ix, g.h[0], g.c0[0]) - q.mu[0];
                const float d1 = fmaf((float)iy, g.h[1], g.c0[1]) - q.mu[1];
                float cb2, cq;
                col_coeffs(q.a00, q.a01, q.a02, q.a11, q.a12, d0, d1, cb2, cq);
                int za, zb;
                if (!col_range(q.a22, cb2, cq, zc, inv_h2, k2, untrunc, q.lo2, q.hi2, za, zb))
                    continue;
                const float *gcol = g_vol + ((int64_t)ix * g.n[1] + iy) * g.n[2];
                float St = 0.0f, Sz = 0.0f, Szz = 0.0f;
                // every voxel of the range is loaded (the range lies in the
                // grid); voxels outside the ellipsoid add exact zeros, so the
                // loop has no branch and successive voxels' loads overlap
                constexpr int UNR = CT == 1 ? 4 : 1;
#pragma unroll UNR
                for (int iz = za; iz <= zb; ++iz) {
                    float gl[CM];
#pragma unroll
                    for (int c = 0; c < CM; ++c)
                        if (c < C) gl[c] = gcol[c * N + iz];
                    const float d2 = fmaf((float)iz, g.h[2], g.c0[2]) - q.mu[2];
                    const float mm = col_quad(q.a22, cb2, cq, d2);
                    const float ev = mm <= k2 ? __expf(-0.5f * mm) : 0.0f;
                    float Gj = 0.0f;
#pragma unroll
                    for (int c = 0; c < CM; ++c) {
                        if (c < C) {
                            gv[c] = fmaf(gl[c], ev, gv[c]);
                            Gj = fmaf(val[c], gl[c], Gj);
                        }
                    }
                    const float t = Gj * ev;
                    St += t;
                    const float td = t * d2;
                    Sz += td;
                    Szz = fmaf(td, d2, Szz);
                }
                P0 = fmaf(d0, St, P0);
                P1 = fmaf(d1, St, P1);
                P2 += Sz;
                M00 = fmaf(d0 * St, d0, M00);
                M01 = fmaf(d0 * St, d1, M01);
                M02 = fmaf(d0, Sz, M02);
                M11 = fmaf(d1 * St, d1, M11);
                M12 = fmaf(d1, Sz, M12);
                M22 += Szz;
            }
        }
#pragma unroll
        for (int c = 0; c < CM; ++c)
            if (c < C) gv[c] = wave_sum_lane63(gv[c]);
        P0 = wave_sum_lane63(P0);
        P1 = wave_sum_lane63(P1);
        P2 = wave_sum_lane63(P2);
        M00 = wave_sum_lane63(M00);
        M01 = wave_sum_lane63(M01);
        M02 = wave_sum_lane63(M02);
        M11 = wave_sum_lane63(M11);
        M12 = wave_sum_lane63(M12);
        M22 = wave_sum_lane63(M22);
        if (lane == 63) {
            float *o = sums[j];
#pragma unroll
            for (int c = 0; c < CM; ++c)
                if (c < C) o[c] = gv[c];
            o[CM + 0] = P0;
            o[CM + 1] = P1;
            o[CM + 2] = P2;
            o[CM + 3] = M00;
            o[CM + 4] = M01;
            o[CM + 5] = M02;
            o[CM + 6] = M11;
            o[CM + 7] = M12;
            o[CM + 8] = M22;
        }
    }
    __syncthreads();
    // chain rule: lane j for Gaussian g0 + j
    const int64_t gi = g0 + lane;
    if (lane >= nj) return;
    const VoxG q = gb[lane];
    if (!(q.lo0 <= q.hi0 && q.lo1 <= q.hi1 && q.lo2 <= q.hi2)) {   // no voxel: zero gradients
        for (int c = 0; c < C; ++c) gr.value[gi * C + c] = 0.0f;
        for (int a = 0; a < 3; ++a) {
            gr.mean[3 * gi + a] = 0.0f;
            gr.scale[3 * gi + a] = 0.0f;
        }
        for (int c = 0; c < 4; ++c) gr.quat[4 * gi + c] = 0.0f;
        return;
    }
    GaussFull G;
    gauss_full(gs.mean, gs.scale, gs.quat, gi, k, g, G);
    const float *o = sums[lane];
    for (int c = 0; c < C; ++c) gr.value[gi * C + c] = o[c];
    const float P[3] = {o[CM + 0], o[CM + 1], o[CM + 2]};
    // mean: d/dmu of -m/2 is A d, so dL/dmu = A sum t d
    for (int a = 0; a < 3; ++a)
        gr.mean[3 * gi + a] = G.A[a][0] * P[0] + G.A[a][1] * P[1] + G.A[a][2] * P[2];
    // d/dA of -m/2 is -d d^T / 2
    const float M[3][3] = {{-0.5f * o[CM + 3], -0.5f * o[CM + 4], -0.5f * o[CM + 5]},
                           {-0.5f * o[CM + 4], -0.5f * o[CM + 6], -0.5f * o[CM + 7]},
                           {-0.5f * o[CM + 5], -0.5f * o[CM + 7], -0.5f * o[CM + 8]}};
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
        // Gaussians per wave: at least ~12,500 waves (a dozen per SIMD) to
        // hide the loads' latency, then as many Gaussians per wave as keeps
        // that (the set-up and the chain rule run lane-parallel over a
        // wave's Gaussians); measured on 200k one-channel and 1k-16k
        // nine-channel sets
        int per = 1;
        const int choice = tune_get(KNOB_VOXELIZE_BWD);
        if (choice > 0)
            per = 1 << (choice - 1);
        else
            while (per < 64 && gs.m / (2 * per) > 12500) per *= 2;
        const unsigned nb = (unsigned)((gs.m + per - 1) / per);
        const int cm = gs.c == 1 || gs.c == 3 || gs.c == 9 ? gs.c : MAXC_VOX;
        const size_t lds = (size_t)per * (sizeof(VoxG) + sizeof(float) * (2 * cm + BW_NS));
        if (gs.c == 1)
            k_vox_bwd<1, false><<<nb, 64, lds, s>>>(gs, g, k, per, g_vol, gr);
        else if (gs.c == 3)
            k_vox_bwd<3, true><<<nb, 64, lds, s>>>(gs, g, k, per, g_vol, gr);
        else if (gs.c == 9)
            k_vox_bwd<9, true><<<nb, 64, lds, s>>>(gs, g, k, per, g_vol, gr);
        else
            k_vox_bwd<0, true><<<nb, 64, lds, s>>>(gs, g, k, per, g_vol, gr);
    }
    return hipGetLastError();
}

}  // namespace pmf
