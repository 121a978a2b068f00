// project.hip -- cone-beam line integrals (Eq. 6) and their exact adjoint.
//
// Forward: one thread per ray (a wave's 64 rays form a tunable pixel tile so
// that they sample neighbouring voxels), midpoint rule in voxel units with
// sample s at u = fma(s, su, bu).
//
// Adjoint: cell-brick owners, no global atomics.  The cells of the grid are
// split into disjoint bricks; a workgroup owns one brick of one view, visits
// every ray of the detector rectangle that bounds the brick's shadow, takes
// exactly the samples whose cell lies in the brick and adds their 8 corner
// weights into an LDS box (the brick's voxels plus a one-voxel pad on the
// high side of each axis) in fixed point.  Each ray's sample positions come
// from one per-ray table, so every brick sees bit-identical samples and no
// sample is lost or counted twice.  Own voxels are stored directly; pads are
// carried to the next brick of a z-chunk or staged, and a fix-up pass adds
// the staged pads into the voxels they belong to in a fixed order.
#include <math.h>

#include <algorithm>

#include "pmf_internal.h"

namespace pmf {

// Per-ray set-up of the midpoint rule, in double precision (a few dozen
// operations per ray against hundreds of samples).  Kept free of FMA
// contraction so every kernel that calls it gets identical bits.
__device__ __forceinline__ RayK ray_setup(const GridK &g, const ConeK &c, double ct,
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


// Branch-free cell coordinate on one axis (same arithmetic as axis_cell):
// fi = clamped cell index as a float, f = fraction; ok = inside the box.
__device__ __forceinline__ void cell_bf(float u, int n, float &fi, float &f, bool &ok) {
    const float nm1 = (float)(n - 1);
    ok = (u >= -0.5f) && (u <= (float)n - 0.5f);
    const float uc = fminf(fmaxf(u, 0.0f), nm1);
    fi = fminf(floorf(uc), nm1 - 1.0f);
    f = uc - fi;
}

// Cell index (as a float) and fraction of a ray sample on one axis.  Ray
// samples are midpoints of the ray's chord through the box, so they lie
// inside it: the coordinate is only clamped (rim voxels take the edge value),
// never rejected -- which also keeps a grazing ray's first sample, that float
// rounding can place a hair outside the box, at its exact-arithmetic value.
__device__ __forceinline__ void ray_cell(float u, float nm1, float nm2, float &fi, float &f) {
    const float uc = __builtin_amdgcn_fmed3f(u, 0.0f, nm1);
    fi = fminf(floorf(uc), nm2);
    f = uc - fi;
}

// Per-grid constants of the ray march: n-1, n-2 per axis and the element
// strides of axes 0 and 1 (24-bit multiplies: n1*n2 < 2^24, N < 2^30).
struct MarchK {
    float nm1[3], nm2[3];
    uint32_t s0, s1;
};

__device__ __forceinline__ float march_sample(const char *__restrict__ vb, const MarchK &mk,
                                              float u0, float u1, float u2) {
    float c0, c1, c2, f0, f1, f2;
    ray_cell(u0, mk.nm1[0], mk.nm2[0], c0, f0);
    ray_cell(u1, mk.nm1[1], mk.nm2[1], c1, f1);
    ray_cell(u2, mk.nm1[2], mk.nm2[2], c2, f2);
    const uint32_t idx =
        __umul24((uint32_t)c0, mk.s0) + __umul24((uint32_t)c1, mk.s1) + (uint32_t)c2;
    const uint32_t o00 = idx * 4u, o01 = o00 + mk.s1 * 4u, o10 = o00 + mk.s0 * 4u,
                   o11 = o10 + mk.s1 * 4u;
    const float *pa = (const float *)(vb + o00), *pb = (const float *)(vb + o01);
    const float *pd = (const float *)(vb + o10), *pe = (const float *)(vb + o11);
    const float x00 = lerp1(pa[0], pa[1], f2), x01 = lerp1(pb[0], pb[1], f2);
    const float x10 = lerp1(pd[0], pd[1], f2), x11 = lerp1(pe[0], pe[1], f2);
    return lerp1(lerp1(x00, x01, f1), lerp1(x10, x11, f1), f0);
}

// The same trilinear read from a y-paired volume: element (i, j, k) holds the
// pair (V[i][j][k], V[i][j+1][k]), so the 2x2 (y, z) corners of a cell are 16
// contiguous bytes and a sample takes two loads (x and x+1) instead of four.
// The blend is the same arithmetic in the same order as march_sample.
__device__ __forceinline__ float march_sample_paired(const char *__restrict__ vb,
                                                     const MarchK &mk, float u0, float u1,
                                                     float u2) {
    float c0, c1, c2, f0, f1, f2;
    ray_cell(u0, mk.nm1[0], mk.nm2[0], c0, f0);
    ray_cell(u1, mk.nm1[1], mk.nm2[1], c1, f1);
    ray_cell(u2, mk.nm1[2], mk.nm2[2], c2, f2);
    const uint32_t idx =
        __umul24((uint32_t)c0, mk.s0) + __umul24((uint32_t)c1, mk.s1) + (uint32_t)c2 * 2u;
    const float *pa = (const float *)(vb + idx * 4u);
    const float *pd = (const float *)(vb + (idx + mk.s0) * 4u);
    // pa[0..3] = V[c0][c1][c2], V[c0][c1+1][c2], V[c0][c1][c2+1], V[c0][c1+1][c2+1]
    const float a0 = pa[0], a1 = pa[1], a2 = pa[2], a3 = pa[3];
    const float d0 = pd[0], d1 = pd[1], d2 = pd[2], d3 = pd[3];
    const float x00 = lerp1(a0, a2, f2), x01 = lerp1(a1, a3, f2);
    const float x10 = lerp1(d0, d2, f2), x11 = lerp1(d1, d3, f2);
    return lerp1(lerp1(x00, x01, f1), lerp1(x10, x11, f1), f0);
}

// a * b + c on the 24-bit multiplier (a, b < 2^24); written out because the
// compiler otherwise masks and takes the full 32-bit multiply here.
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Samples whose coordinates lie in (0, n-1) on every axis need none of
// ray_cell's clamps: the cell index is the truncation and the fraction
// u - floor(u) is exact for u >= 0 (what v_fract returns), so the two reads
// below give the same bits as march_sample / march_sample_paired with fewer
// operations (no clamps, no float floors to convert).
__device__ __forceinline__ float march_body(const char *__restrict__ vb, const MarchK &mk,
                                            float u0, float u1, float u2) {
    const float f0 = __builtin_amdgcn_fractf(u0), f1 = __builtin_amdgcn_fractf(u1),
                f2 = __builtin_amdgcn_fractf(u2);
    const uint32_t o00 =
        mad_u24((uint32_t)u0, mk.s0, mad_u24((uint32_t)u1, mk.s1, (uint32_t)u2)) * 4u;
    const uint32_t o01 = o00 + mk.s1 * 4u, o10 = o00 + mk.s0 * 4u, o11 = o10 + mk.s1 * 4u;
    const float *pa = (const float *)(vb + o00), *pb = (const float *)(vb + o01);
    const float *pd = (const float *)(vb + o10), *pe = (const float *)(vb + o11);
    const float x00 = lerp1(pa[0], pa[1], f2), x01 = lerp1(pb[0], pb[1], f2);
    const float x10 = lerp1(pd[0], pd[1], f2), x11 = lerp1(pe[0], pe[1], f2);
    return lerp1(lerp1(x00, x01, f1), lerp1(x10, x11, f1), f0);
}

// Byte offset of a body sample's cell in the y-paired layout.
__device__ __forceinline__ uint32_t body_offset_paired(const MarchK &mk, float u0, float u1,
                                                       float u2) {
    return mad_u24((uint32_t)u0, mk.s0, mad_u24((uint32_t)u1, mk.s1, (uint32_t)u2 * 2u)) * 4u;
}

__device__ __forceinline__ float march_body_paired(const char *__restrict__ vb,
                                                   const MarchK &mk, float u0, float u1,
                                                   float u2) {
    const float f0 = __builtin_amdgcn_fractf(u0), f1 = __builtin_amdgcn_fractf(u1),
                f2 = __builtin_amdgcn_fractf(u2);
    const uint32_t o = body_offset_paired(mk, u0, u1, u2);
    const float *pa = (const float *)(vb + o);
    const float *pd = (const float *)(vb + (o + mk.s0 * 4u));
    const float a0 = pa[0], a1 = pa[1], a2 = pa[2], a3 = pa[3];
    const float d0 = pd[0], d1 = pd[1], d2 = pd[2], d3 = pd[3];
    const float x00 = lerp1(a0, a2, f2), x01 = lerp1(a1, a3, f2);
    const float x10 = lerp1(d0, d2, f2), x11 = lerp1(d1, d3, f2);
    return lerp1(lerp1(x00, x01, f1), lerp1(x10, x11, f1), f0);
}

// The samples [sb, se) of a ray whose coordinates lie in [1/64, n-1-1/64] on
// every axis (so march_body applies).  The crossing indices are estimated in
// float with a 1/64-sample guard; their error, below 1e-4 voxel in
// coordinate terms, cannot carry a sample from inside the margin to outside
// (0, n-1).
__device__ __forceinline__ void body_range(const RayK &r, const MarchK &mk, int &sb, int &se) {
    constexpr float M = 0.015625f;
    float lo = 0.0f, hi = (float)r.n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float xl = M, xh = mk.nm1[a] - M, su = r.su[a], bu = r.bu[a];
        if (su == 0.0f) {
            if (!(bu >= xl && bu <= xh)) hi = -1.0f;
        } else {
            const float t1 = (xl - bu) / su, t2 = (xh - bu) / su;
            lo = fmaxf(lo, fminf(t1, t2));
            hi = fminf(hi, fmaxf(t1, t2));
        }
    }
    lo = fminf(lo, (float)r.n);
    hi = fmaxf(hi, -1.0f);
    sb = (int)ceilf(lo + M);
    se = max((int)floorf(hi - M) + 1, sb);
}

__host__ __device__ inline MarchK make_march(const GridK &g) {
    MarchK m;
    for (int a = 0; a < 3; ++a) {
        m.nm1[a] = (float)(g.n[a] - 1);
        m.nm2[a] = (float)(g.n[a] - 2);
    }
    m.s1 = (uint32_t)g.n[2];
    m.s0 = (uint32_t)g.n[1] * (uint32_t)g.n[2];
    return m;
}

// Strides (elements) of the y-paired layout: two floats per voxel.
__host__ __device__ inline MarchK make_march_paired(const GridK &g) {
    MarchK m = make_march(g);
    m.s1 *= 2u;
    m.s0 *= 2u;
    return m;
}

// Forward pixel tiles: a wave takes WU x WV pixels (u x v), the four waves of
// a workgroup sit AU across and 4/AU down.  The wave's footprint decides how
// many distinct cache lines each of its gathers touches: v runs along z, the
// fastest (contiguous) axis of the volume, so narrow-and-tall wave tiles touch
// fewer lines per load.
//
// One launch serves up to MAXS scans (a ragged batch): workgroups
// [first[k], first[k+1]) belong to scan k, view-major, tiles row-major.
struct ProjK {
    const float *vol;
    int64_t stride;
    GridK g;
    ConeK c;
    MarchK mk;
    const float *angles;
    float *proj;
    int tiles_u, ntiles;
    int items;              // ntiles * V
};
struct ProjTab {
    ProjK s[MAXS];
    int first[MAXS + 1];
    int n;
};

template <int WU, int WV, int AU, bool PAIRED>
__global__ __launch_bounds__(256) void k_project(ProjTab t) {
    static_assert(WU * WV == 64 && AU >= 1 && 4 % AU == 0, "wave tile must hold 64 pixels");
    constexpr int BU = WU * AU, BV = WV * (4 / AU);
    // within each scan, each XCD takes one contiguous range of its (view,
    // tile) items: whole views and neighbouring tiles share an L2 (measured
    // faster than sharing each view across all XCDs), and every XCD gets an
    // equal share of every scan
    const int job = job_of(t, (int)blockIdx.x);
    const ProjK &pj = t.s[job];
    const int local = job_item(t, job, (int)blockIdx.x);
    if (local >= pj.items) return;
    const GridK &g = pj.g;
    const ConeK &c = pj.c;
    const MarchK &mk = pj.mk;
    const int v = local / pj.ntiles, tile = local - v * pj.ntiles;
    const int tu = tile % pj.tiles_u, tv = tile / pj.tiles_u;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int iu = tu * BU + (w % AU) * WU + l % WU;
    const int iv = tv * BV + (w / AU) * WV + l / WU;
    if (iu >= c.nu || iv >= c.nv) return;
    const double th = (double)pj.angles[v];
    const RayK r = ray_setup(g, c, cos(th), sin(th), iu, iv);
    const char *__restrict__ vb = (const char *)(pj.vol + (int64_t)v * pj.stride);
    float acc0 = 0.0f, acc1 = 0.0f;
    auto sample = [&](float sf) {
        const float u0 = fmaf(sf, r.su[0], r.bu[0]), u1 = fmaf(sf, r.su[1], r.bu[1]),
                    u2 = fmaf(sf, r.su[2], r.bu[2]);
        return PAIRED ? march_sample_paired(vb, mk, u0, u1, u2) : march_sample(vb, mk, u0, u1, u2);
    };
    auto body = [&](float sf) {
        const float u0 = fmaf(sf, r.su[0], r.bu[0]), u1 = fmaf(sf, r.su[1], r.bu[1]),
                    u2 = fmaf(sf, r.su[2], r.bu[2]);
        return PAIRED ? march_body_paired(vb, mk, u0, u1, u2) : march_body(vb, mk, u0, u1, u2);
    };
    // clamped head, unclamped body in pairs, clamped tail (a fixed order per
    // ray whatever the launch shape)
    int sb, se;
    body_range(r, mk, sb, se);
    sb = min(sb, r.n);
    se = min(se, r.n);
    int s = 0;
    for (; s < sb; ++s) acc0 += sample((float)s);
    if constexpr (PAIRED) {
        // Consecutive samples of a ray often share a cell: a lane reloads its
        // eight corners only when the cell changes, which takes that lane out
        // of the gather (the loads are the limit here, not the arithmetic).
        uint32_t last = 0xffffffffu;
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, d0 = 0.0f, d1 = 0.0f, d2 = 0.0f,
              d3 = 0.0f;
        float sf = (float)s;
        for (; s < se; ++s, sf += 1.0f) {
            const float u0 = fmaf(sf, r.su[0], r.bu[0]), u1 = fmaf(sf, r.su[1], r.bu[1]),
                        u2 = fmaf(sf, r.su[2], r.bu[2]);
            const uint32_t o = body_offset_paired(mk, u0, u1, u2);
            if (o != last) {
                const float *pa = (const float *)(vb + o);
                const float *pd = (const float *)(vb + (o + mk.s0 * 4u));
                a0 = pa[0]; a1 = pa[1]; a2 = pa[2]; a3 = pa[3];
                d0 = pd[0]; d1 = pd[1]; d2 = pd[2]; d3 = pd[3];
                last = o;
            }
            const float f0 = __builtin_amdgcn_fractf(u0), f1 = __builtin_amdgcn_fractf(u1),
                        f2 = __builtin_amdgcn_fractf(u2);
            const float x00 = lerp1(a0, a2, f2), x01 = lerp1(a1, a3, f2);
            const float x10 = lerp1(d0, d2, f2), x11 = lerp1(d1, d3, f2);
            acc1 += lerp1(lerp1(x00, x01, f1), lerp1(x10, x11, f1), f0);
        }
    } else {
        float sf = (float)s;
        for (; s + 1 < se; s += 2, sf += 2.0f) {
            acc0 += body(sf);
            acc1 += body(sf + 1.0f);
        }
    }
    for (; s < r.n; ++s) acc0 += sample((float)s);
    pj.proj[((int64_t)v * c.nv + iv) * c.nu + iu] = (acc0 + acc1) * r.delta;
}

// Per-ray constants of every view, per view the brick orientation of the
// back-projection, and per view the two figures that set its fixed-point
// scale: the largest |g_proj * delta| over the
// rays, and the smallest step over the rays with at least two samples (a ray
// with one sample gives any voxel at most one contribution).  The grid is
// (workgroups per view, V): a workgroup strides over the rays of one view and
// adds its two figures with one atomic each.
__global__ __launch_bounds__(256) void k_ray_table(GridK g, ConeK c,
                                                   const float *__restrict__ angles,
                                                   const float *__restrict__ g_proj,
                                                   RayK *__restrict__ out,
                                                   unsigned *__restrict__ stats,
                                                   int *__restrict__ orient) {
    __shared__ float red[8];
    const int npix = c.nu * c.nv;
    const int v = blockIdx.y;
    const double th = (double)angles[v];
    const double ct = cos(th), st = sin(th);
    // the back-projection's brick orientation: long edge along axis 1 when
    // the view's rays run mostly along it
    if (blockIdx.x == 0 && threadIdx.x == 0) orient[v] = fabs(st) > fabs(ct) ? 1 : 0;
    float m = 0.0f, d = INFINITY;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += gridDim.x * blockDim.x) {
        const RayK r = ray_setup(g, c, ct, st, p % c.nu, p / c.nu);
        const int64_t q = (int64_t)v * npix + p;
        out[q] = r;
        if (r.n > 0) m = fmaxf(m, fabsf(g_proj[q] * r.delta));
        if (r.n > 1) d = fminf(d, r.delta);
    }
    for (int o = 32; o > 0; o >>= 1) {
        m = fmaxf(m, __shfl_xor(m, o, 64));
        d = fminf(d, __shfl_xor(d, o, 64));
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wave] = m;
        red[4 + wave] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        d = fminf(fminf(red[4], red[5]), fminf(red[6], red[7]));
        // non-negative floats order like their bit patterns
        if (m > 0.0f) atomicMax(&stats[2 * v], __float_as_uint(m));
        if (d < INFINITY) atomicMin(&stats[2 * v + 1], __float_as_uint(d));
    }
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


// Round to the nearest integer (halves up) in one instruction.
__device__ __forceinline__ int round_int(float x) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// acc = acc * k + e, written in place (keeps a loop-carried accumulator in
// its register instead of a copy per iteration).
__device__ __forceinline__ void fma_in_place(float &acc, float k, float e) {
    asm("v_fma_f32 %0, %0, %1, %2" : "+v"(acc) : "v"(k), "v"(e));
}

// 0.0 in the lanes set in mask, 1.0 in the others (one select on the mask's
// SGPR pair, so a compare feeding both a branch and this needs no twin).
__device__ __forceinline__ float zero_where(unsigned long long mask) {
    float r;
    asm("v_cndmask_b32_e64 %0, 1.0, 0, %1" : "=v"(r) : "s"(mask));
    return r;
}

// Waits for this wave's outstanding LDS reads (and, LDS operations retiring
// in order, everything issued before them).  Placed right after the rare
// reads of a ray switch so the compiler need not put a conservative wait on
// the common path, where it would also wait for the previous sample's
// atomics.
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0xc07f); }  // lgkmcnt(0)

// One ray's owned run, staged in LDS for the lanes that take its samples:
// item q of the wave's flattened list is sample q + off of the ray.
struct RunP {
    float bu[3], su[3], gp;
    int off;
};


struct BoundK {
    float mag, persp, R, Z, two_hx, two_hy, two_hz, inv_du, inv_dv, diag;
};

// The adjoint of the ray march, g_vol_v = P_v^T g_proj, by brick owners.
//
// Ownership: the cells (i, i+1 per axis) of the grid are split into disjoint
// bricks of S0 x S1 x S2 cells; a workgroup owns one brick of one view and
// takes exactly the samples whose cell lies in it, so every sample is
// scattered once.  Its 8 corner weights land in an LDS box of (S+1) voxels
// per axis: the brick's own voxels and a one-voxel pad on the high side of
// each axis, which belongs to the next brick.  Own voxels are stored to
// g_vol directly.  A workgroup walks a chunk of bricks along axis 2 and
// carries each brick's axis-2 pad layer in LDS into the next brick (those
// voxels are contiguous in memory only along axis 2, so staging them would
// cost a cache line per voxel); the other pads are staged per (view, brick)
// and a fix-up pass adds them into the voxels they belong to, in a fixed
// order.
//
// Shape: a brick is long (L cells) along the horizontal axis the view's rays
// mostly follow and W cells across it (H along z), so a ray's run in one
// brick is long and its set-up (reading its constants, finding the run) is
// spread over many samples.  Every brick of a view has the same orientation.
//
// Work distribution: each wave takes 64 rays of the brick's detector shadow
// at a time (an 8x8 grid of pixels spread over the shadow rectangle), finds
// each ray's run of owned samples, and flattens the runs into one list of
// (ray, sample) items by a prefix sum over the lanes; each lane then walks
// an equal slice of that list, so every lane does a sample per iteration
// however the run lengths differ, and the lanes of a wave stay in different
// rays (their LDS atomics seldom hit the same word).
//
// Accumulation is in 32-bit fixed point with integer LDS atomics, so the
// sums do not depend on their order.  For each view the scale is
// 2^30 / (kbound * M), where M is the largest |g_proj * delta| among the
// view's rays and kbound bounds how many samples can touch one voxel in this
// view (from the geometry and the smallest step of the rays with two or more
// samples): every sum stays below 2^30 in magnitude, and each contribution
// is rounded to within 0.5 / scale.  Optionally (MERGE) a lane adds
// consecutive samples that fall in one cell in registers and rounds their
// sum once, which saves LDS traffic but not instructions.  The scale is the
// same in every brick of a view, so a pad and the voxel it belongs to add up
// as partial sums of one fixed-point sum.  With vmax non-null the largest
// |g_vol| of each view is recorded (by the fix-up for the voxels it
// completes).

// One scan's share of a ragged back-projection launch: workgroups
// [first[k], first[k+1]) belong to scan k, view-major (nbv items per view,
// the brick count of the orientation with more bricks) or one per brick when
// summing over views.
struct BwdK {
    const float *g_proj;
    GridK g;
    ConeK c;
    const float *angles;
    const RayK *rays;
    const unsigned *stats;
    const int *orient;      // [V]: 1 when the view's rays run mostly along axis 1
    int V;
    float *g_vol;
    int64_t stride;
    float *pads;            // [V (or 1)][nbb][NPMAX]: one box per brick
    int nbb;                // bricks per view (the orientation with more)
    int zc;                 // bricks per chunk along axis 2 (per-view mode)
    int nbv;                // work items per view (column chunks, or bricks when summing)
    int items;              // nbv * V, or nbv when summing over views
    BoundK kb;
    MarchK mk;
    unsigned *vmax;
};
struct BwdTab {
    BwdK s[MAXS];
    int first[MAXS + 1];
    int n;
};

// Geometry of one brick: owned cells [clo, chi] per axis, their extent in
// voxel units [ulo, uhi] and world box [wlo, whi], and whether every owned
// cell avoids the clamped rim cells.
struct BrickGeo {
    int B[3];
    float clo[3], chi[3], ulo[3], uhi[3];
    double wlo[3], whi[3];
    bool interior, cells;
};

template <int S0, int S1, int S2>
__device__ __forceinline__ BrickGeo brick_geo(const GridK &g, int b0, int b1, int b2) {
    constexpr int SZ[3] = {S0, S1, S2};
    BrickGeo q;
    q.B[0] = b0 * S0;
    q.B[1] = b1 * S1;
    q.B[2] = b2 * S2;
    q.interior = true;
    q.cells = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int lo = q.B[a], hi = min(q.B[a] + SZ[a] - 1, g.n[a] - 2);
        q.cells = q.cells && lo <= hi;
        q.clo[a] = (float)lo;
        q.chi[a] = (float)hi;
        q.interior = q.interior && lo >= 1 && hi <= g.n[a] - 3;
        q.ulo[a] = lo == 0 ? -0.5f : (float)lo;
        q.uhi[a] = hi == g.n[a] - 2 ? (float)g.n[a] - 0.5f : (float)(hi + 1);
        q.wlo[a] = g.c0d[a] + ((double)q.ulo[a] - 0.5) * g.hd[a];
        q.whi[a] = g.c0d[a] + ((double)q.uhi[a] + 0.5) * g.hd[a];
    }
    return q;
}

// Fixed-point scale of view v: 2^30 / (kbound M) (see above); 0 when the view
// has no residual.
__device__ __forceinline__ float bp_scale(const BwdK &bj, int v, double ct, double st) {
    const BoundK &kb = bj.kb;
    const float m = __uint_as_float(bj.stats[2 * v]);
    const float dmin = __uint_as_float(bj.stats[2 * v + 1]);
    if (!(m > 0.0f)) return 0.0f;
    // Contributions one voxel can receive in this view: rays through the
    // detector shadow of its 2x2x2-cell support, times samples of one ray
    // inside that support (its diagonal over the smallest step, plus one).
    const float as = fabsf((float)st), ac = fabsf((float)ct);
    const float lat = kb.two_hx * as + kb.two_hy * ac;    // lateral extent (mm)
    const float dep = kb.two_hx * ac + kb.two_hy * as;    // depth extent (mm)
    const float wu = lat * kb.mag + kb.R * kb.persp * dep;
    const float wv = kb.two_hz * kb.mag + kb.Z * kb.persp * dep;
    const float nr = (floorf(wu * kb.inv_du) + 1.0f) * (floorf(wv * kb.inv_dv) + 1.0f);
    const float ns = floorf(kb.diag / dmin) + 1.0f;     // 1 when no ray has two samples
    const float kbound = nr * ns * 1.0625f + 1.0f;
    return 1073741824.0f / (kbound * m);                // 2^30 / (kbound M)
}

// Scatter every owned sample of view v into the LDS box acc (fixed point,
// scale `scale`) of the brick q.  Waves work independently; the caller
// synchronises the workgroup before and after.
template <int S0, int S1, int S2, int NW, bool MERGE>
__device__ __forceinline__ void bp_scatter(const BwdK &bj, const BrickGeo &q, int v, double ct,
                                           double st, float scale, int *__restrict__ acc,
                                           RunP (*__restrict__ runs)[64],
                                           int (*__restrict__ ends)[64]) {
    constexpr int P1 = S1 + 1, P2 = S2 + 1;
    const ConeK &c = bj.c;
    const MarchK &mk = bj.mk;
    const float *__restrict__ g_proj = bj.g_proj;
    const RayK *__restrict__ rays = bj.rays;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wave
    const int lx = lane & 7, ly = lane >> 3;
    // clamp limits of the rim path, held in registers (a reload from the
    // argument table inside the sample loop would also wait for the atomics)
    float nm1[3], nm2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nm1[a] = mk.nm1[a];
        nm2[a] = mk.nm2[a];
        asm volatile("" : "+s"(nm1[a]), "+s"(nm2[a]));
    }
    const bool interior = q.interior;
    // byte offset in acc of cell (c0, c1, c2): c0*K0 + c1*K1 + c2*4 + KC,
    // exact in float (every term is an integer below 2^24)
    const float K0 = 4.0f * P1 * P2, K1 = 4.0f * P2;
    const float KC = -4.0f * ((float)q.B[0] * P1 * P2 + (float)q.B[1] * P2 + (float)q.B[2]);
    int u0, u1, v0, v1;
    shadow_rect(c, ct, st, q.wlo, q.whi, u0, u1, v0, v1);   // uniform across the block
    if (u1 < u0 || v1 < v0) return;
    // The 64 lanes of a wave take an 8x8 grid of pixels spread over the
    // rectangle (strides gu, gv); the waves sweep the gu*gv offsets.  Rays
    // that far apart keep the lanes' LDS atomics on unrelated words.
    const int gu = (u1 - u0 + 8) / 8, gv = (v1 - v0 + 8) / 8;
    const int nph = gu * gv;
    RunP *const wr = runs[wave];
    int *const we = ends[wave];
    for (int ph = wave; ph < nph; ph += NW) {            // uniform per wave
        const int iu = u0 + lx * gu + ph % gu, iv = v0 + ly * gv + ph / gu;
        int s0 = 0, len = 0;
        RayK r;
        float gp = 0.0f;
        if (iu <= u1 && iv <= v1) {
            const int64_t pix = ((int64_t)v * c.nv + iv) * c.nu + iu;
            r = rays[pix];
            gp = g_proj[pix] * r.delta * scale;
            if (r.n > 0 && gp != 0.0f) {
                float smin = 0.0f, smax = (float)(r.n - 1);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (r.su[a] != 0.0f) {
                        // an estimate only: the run is made exact below
                        const float inv = __builtin_amdgcn_rcpf(r.su[a]);
                        const float ta = (q.ulo[a] - r.bu[a]) * inv, tb = (q.uhi[a] - r.bu[a]) * inv;
                        smin = fmaxf(smin, fminf(ta, tb));
                        smax = fminf(smax, fmaxf(ta, tb));
                    } else if (r.bu[a] < q.ulo[a] - 1.0f || r.bu[a] > q.uhi[a] + 1.0f) {
                        smax = -10.0f;
                    }
                }
                if (smin <= smax + 2.0f) {
                    // The owned samples form one run of s: every axis's cell
                    // index is monotone in s and the owned cells form a box.
                    // The estimate puts the run at [ceil(smin), ceil(smax) - 1]
                    // up to rounding far below one sample; start one sample
                    // outside each end and move to the exact ends.
                    // (in an interior brick the clamps cannot change the
                    // answer: owned cells lie in [1, n-3] on every axis)
                    auto cell = [&](float x, int a) {
                        if (interior) return floorf(x);
                        float fi, fr;
                        ray_cell(x, nm1[a], nm2[a], fi, fr);
                        return fi;
                    };
                    auto owned = [&](int si) {
                        const float sf = (float)si;
                        if (interior) {
                            // floor(x) in [clo, chi] <=> clo <= x < chi + 1,
                            // and ulo = clo, uhi = chi + 1 in an interior brick
                            const float x0 = fmaf(sf, r.su[0], r.bu[0]);
                            const float x1 = fmaf(sf, r.su[1], r.bu[1]);
                            const float x2 = fmaf(sf, r.su[2], r.bu[2]);
                            return x0 >= q.ulo[0] && x0 < q.uhi[0] && x1 >= q.ulo[1] &&
                                   x1 < q.uhi[1] && x2 >= q.ulo[2] && x2 < q.uhi[2];
                        }
                        float fi = cell(fmaf(sf, r.su[0], r.bu[0]), 0);
                        bool o = fi >= q.clo[0] && fi <= q.chi[0];
                        fi = cell(fmaf(sf, r.su[1], r.bu[1]), 1);
                        o = o && fi >= q.clo[1] && fi <= q.chi[1];
                        fi = cell(fmaf(sf, r.su[2], r.bu[2]), 2);
                        return o && fi >= q.clo[2] && fi <= q.chi[2];
                    };
                    const int last = r.n - 1;
                    s0 = min(max(0, (int)ceilf(smin) - 1), last);
                    int s1 = min(max(0, (int)ceilf(smax)), last);
                    bool found;
                    if (owned(s0)) {
                        while (s0 > 0 && owned(s0 - 1)) --s0;
                        found = true;
                    } else {
                        ++s0;
                        while (s0 <= s1 && !owned(s0)) ++s0;
                        found = s0 <= s1;
                    }
                    if (found) {
                        s1 = max(s1, s0);
                        if (owned(s1)) {
                            while (s1 < last && owned(s1 + 1)) ++s1;
                        } else {
                            --s1;
                            while (s1 > s0 && !owned(s1)) --s1;
                        }
                        len = s1 - s0 + 1;
                    }
                }
            }
        }
        // flatten the wave's runs: item q in [start, start + len) is
        // sample q - start + s0 of this lane's ray.  Only non-empty runs are
        // stored (compacted in lane order), so a lane's walk crosses from
        // one run to the next in one step; the ends past the last run hold
        // T for the search below.
        const int incl = wave_incl_sum(len);
        const int T = __builtin_amdgcn_readlane(incl, 63);
        if (T == 0) continue;
        {
            const unsigned long long nz = __ballot(len > 0);
            const int pos = __builtin_amdgcn_mbcnt_hi((unsigned)(nz >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)nz, 0u));
            const int NR = __popcll(nz);
            RunP rp;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                rp.bu[a] = r.bu[a];
                rp.su[a] = r.su[a];
            }
            rp.gp = gp;
            rp.off = s0 - (incl - len);
            if (len > 0) {
                wr[pos] = rp;
                we[pos] = incl;
            }
            if (lane >= NR) we[lane] = T;
        }
        wave_lds_sync();
        // Lane j takes items [j K, j K + K): every lane does a sample per
        // step however the run lengths differ.
        const int K = (T + 63) >> 6;
        int it = lane * K;
        const int ite = min(it + K, T);
        // first run of the slice: the smallest r with end_r > it (binary
        // lifting)
        int ri = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (we[ri + step - 1] <= it) ri += step;
        int rend = we[ri];
        RunP rp = wr[ri];
        lds_wait();
        // Sample s of ray rp: its cell's LDS byte offset and the 8 corner
        // weights.
        auto sample = [&](float sf, int &off, float e[8]) {
            const float x0 = fmaf(sf, rp.su[0], rp.bu[0]);
            const float x1 = fmaf(sf, rp.su[1], rp.bu[1]);
            const float x2 = fmaf(sf, rp.su[2], rp.bu[2]);
            float c0f, c1f, c2f, f0, f1, f2;
            if (interior) {
                c0f = floorf(x0);
                c1f = floorf(x1);
                c2f = floorf(x2);
                f0 = x0 - c0f;
                f1 = x1 - c1f;
                f2 = x2 - c2f;
            } else {
                ray_cell(x0, nm1[0], nm2[0], c0f, f0);
                ray_cell(x1, nm1[1], nm2[1], c1f, f1);
                ray_cell(x2, nm1[2], nm2[2], c2f, f2);
            }
            off = (int)fmaf(c0f, K0, fmaf(c1f, K1, fmaf(c2f, 4.0f, KC)));
            const float w = rp.gp;
            const float wx1 = w * f0, wx0 = w - wx1;
            const float a01 = wx0 * f1, a00 = wx0 - a01;
            const float a11 = wx1 * f1, a10 = wx1 - a11;
            const float e001 = a00 * f2, e011 = a01 * f2;
            const float e101 = a10 * f2, e111 = a11 * f2;
            e[0] = a00 - e001;
            e[1] = e001;
            e[2] = a01 - e011;
            e[3] = e011;
            e[4] = a10 - e101;
            e[5] = e101;
            e[6] = a11 - e111;
            e[7] = e111;
        };
        auto add8 = [&](int off, const float e[8]) {
            char *qb = (char *)acc + off;
            atomicAdd((int *)qb, round_int(e[0]));
            atomicAdd((int *)(qb + 4), round_int(e[1]));
            atomicAdd((int *)(qb + 4 * P2), round_int(e[2]));
            atomicAdd((int *)(qb + 4 * P2 + 4), round_int(e[3]));
            atomicAdd((int *)(qb + 4 * P1 * P2), round_int(e[4]));
            atomicAdd((int *)(qb + 4 * P1 * P2 + 4), round_int(e[5]));
            atomicAdd((int *)(qb + 4 * P1 * P2 + 4 * P2), round_int(e[6]));
            atomicAdd((int *)(qb + 4 * P1 * P2 + 4 * P2 + 4), round_int(e[7]));
        };
        if (!MERGE) {
            // every sample's 8 corners go to LDS at once
            float sf = (float)(it + rp.off);
            for (; it < ite; ++it, sf += 1.0f) {
                if (it >= rend) {           // the next run (none is empty)
                    rend = we[++ri];
                    rp = wr[ri];
                    lds_wait();
                    sf = (float)(it + rp.off);
                }
                int off;
                float e[8];
                sample(sf, off, e);
                add8(off, e);
            }
        } else if (it < ite) {
            // Consecutive samples in one cell add up in registers; the
            // cell's 8 corners go to LDS when the lane moves on.
            int cur_off;
            float cw[8];
            float sf = (float)(it + rp.off);
            sample(sf, cur_off, cw);
            for (++it; it < ite; ++it) {
                sf += 1.0f;                 // exact: sample indices are small integers
                if (it >= rend) {           // the next run (none is empty)
                    rend = we[++ri];
                    rp = wr[ri];
                    lds_wait();
                    sf = (float)(it + rp.off);
                }
                int off;
                float e[8];
                sample(sf, off, e);
                // a restart is a multiply by 0, so both cases share one fma;
                // the factor comes from the branch's own lane mask
                const bool moved = off != cur_off;
                const float keep = zero_where(__ballot(moved));
                if (moved) add8(cur_off, cw);
                cur_off = off;
#pragma unroll
                for (int k = 0; k < 8; ++k) fma_in_place(cw[k], keep, e[k]);
            }
            add8(cur_off, cw);
        }
        wave_lds_sync();
    }
}

// Per-view mode: one workgroup walks a chunk of up to ZC bricks along
// axis 2 of one (b0, b1) column for one view.  The high pad layer of each
// brick (z = S2 in its box) is the low layer of the next one: it is carried
// in LDS (integer sums: exact), so only the chunk's last brick stages it.
// Own voxels go to g_vol, the pads of axes 0 and 1 to the staging box; a
// voxel on a low face whose lower neighbour stages a pad is completed by the
// fix-up (which also takes its part of vmax).
template <int S0, int S1, int S2, int NW, int NPMAX, bool MERGE, int ZC>
__device__ __forceinline__ void bp_column(const BwdK &bj, int view, int item, int *__restrict__ acc,
                                          RunP (*__restrict__ runs)[64],
                                          int (*__restrict__ ends)[64]) {
    constexpr int P1 = S1 + 1, P2 = S2 + 1;
    constexpr int NP = (S0 + 1) * P1 * P2;
    static_assert(NP <= NPMAX, "box larger than the LDS array");
    constexpr int NT = 64 * NW;
    const GridK &g = bj.g;
    const int nb0 = (g.n[0] + S0 - 1) / S0, nb1 = (g.n[1] + S1 - 1) / S1;
    const int nb2 = (g.n[2] + S2 - 1) / S2;
    constexpr int zc = ZC;
    const int nzc = (nb2 + zc - 1) / zc;
    if (item >= nb0 * nb1 * nzc) return;      // the other orientation has more items
    const int chunk = item % nzc, col = item / nzc;
    const int b1 = col % nb1, b0 = col / nb1;
    const int z0 = chunk * zc, z1 = min(nb2, z0 + zc);
    const int v = view;
    const double th = (double)bj.angles[v];
    const double ct = cos(th), st = sin(th);
    const float scale = bp_scale(bj, v, ct, st);
    const float inv_scale = scale > 0.0f ? 1.0f / scale : 0.0f;
    float *out = bj.g_vol + (int64_t)v * bj.stride;
    const int lane = threadIdx.x & 63;
    float mx = 0.0f;
    for (int i = threadIdx.x; i < NP; i += NT) acc[i] = 0;
    __syncthreads();
    for (int b2 = z0; b2 < z1; ++b2) {
        const BrickGeo q = brick_geo<S0, S1, S2>(g, b0, b1, b2);
        if (q.cells && scale > 0.0f) bp_scatter<S0, S1, S2, NW, MERGE>(bj, q, v, ct, st, scale, acc, runs, ends);
        __syncthreads();
        const bool lastb = b2 + 1 == z1;
        float *pad = bj.pads + ((int64_t)v * bj.nbb + (b0 * nb1 + b1) * nb2 + b2) * NPMAX;
        // Row owners: a thread takes one (x, y) row of the box (P2 entries
        // along z), stores it, and then carries its z = S2 entry to z = 0
        // and clears the rest for the next brick (its own row only, so no
        // other thread's reads are in the way).
        const bool zfix = b2 == z0 && b2 > 0;     // the z = 0 layer is completed by the fix-up
        const bool full_z = q.B[2] + S2 <= g.n[2] && (g.n[2] & 3) == 0;
#pragma unroll 1
        for (int r = threadIdx.x; r < (S0 + 1) * P1; r += NT) {
            const int x = r / P1, y = r - x * P1;
            const int gx = q.B[0] + x, gy = q.B[1] + y;
            int *row = acc + r * P2;
            int raw[P2];
#pragma unroll
            for (int z = 0; z < P2; ++z) raw[z] = row[z];
            if (gx < g.n[0] && gy < g.n[1]) {
                float val[P2];
#pragma unroll
                for (int z = 0; z < P2; ++z) val[z] = (float)raw[z] * inv_scale;
                float *orow = out + ((int64_t)gx * g.n[1] + gy) * g.n[2] + q.B[2];
                if (x < S0 && y < S1) {
                    if constexpr (S2 % 4 == 0) {
                        if (full_z && ((uintptr_t)orow & 15) == 0) {
#pragma unroll
                            for (int z = 0; z < S2; z += 4)
                                *(float4 *)(orow + z) = make_float4(val[z], val[z + 1], val[z + 2], val[z + 3]);
                        } else {
#pragma unroll
                            for (int z = 0; z < S2; ++z)
                                if (q.B[2] + z < g.n[2]) orow[z] = val[z];
                        }
                    } else {
#pragma unroll
                        for (int z = 0; z < S2; ++z)
                            if (q.B[2] + z < g.n[2]) orow[z] = val[z];
                    }
                    if (!((x == 0 && b0 > 0) || (y == 0 && b1 > 0))) {
#pragma unroll
                        for (int z = 0; z < S2; ++z)
                            if (q.B[2] + z < g.n[2] && !(z == 0 && zfix)) mx = fmaxf(mx, fabsf(val[z]));
                    }
                    if (lastb && q.B[2] + S2 < g.n[2]) pad[r * P2 + S2] = val[S2];
                } else {
#pragma unroll
                    for (int z = 0; z < P2; ++z)
                        if (q.B[2] + z < g.n[2] && (z < S2 || lastb)) pad[r * P2 + z] = val[z];
                }
            }
            if (!lastb) {
                row[0] = raw[S2];
#pragma unroll
                for (int z = 1; z < P2; ++z) row[z] = 0;
            }
        }
        __syncthreads();
    }
    if (bj.vmax) {
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        if (lane == 0 && mx > 0.0f) atomicMax(&bj.vmax[v], __float_as_uint(mx));
    }
}

// Summed over views: one brick per workgroup (chunks of one brick), every
// view in order with its own scale, float sums per box entry; all pads are
// staged.
template <int S0, int S1, int S2, int NW, int NPMAX, bool MERGE>
__device__ __forceinline__ void bp_summed(const BwdK &bj, int bid, int *__restrict__ acc,
                                          RunP (*__restrict__ runs)[64],
                                          int (*__restrict__ ends)[64]) {
    constexpr int P1 = S1 + 1, P2 = S2 + 1;
    constexpr int NP = (S0 + 1) * P1 * P2;
    static_assert(NP <= NPMAX, "box larger than the LDS array");
    constexpr int NT = 64 * NW;
    constexpr int PER = (NP + NT - 1) / NT;
    const GridK &g = bj.g;
    const int nb0 = (g.n[0] + S0 - 1) / S0, nb1 = (g.n[1] + S1 - 1) / S1;
    const int nb2 = (g.n[2] + S2 - 1) / S2;
    if (bid >= nb0 * nb1 * nb2) return;
    const int b2 = bid % nb2, b1 = (bid / nb2) % nb1, b0 = bid / (nb2 * nb1);
    const BrickGeo q = brick_geo<S0, S1, S2>(g, b0, b1, b2);
    float sum[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) sum[k] = 0.0f;
    for (int v = 0; v < bj.V; ++v) {
        const double th = (double)bj.angles[v];
        const double ct = cos(th), st = sin(th);
        const float scale = bp_scale(bj, v, ct, st);
        if (!q.cells || !(scale > 0.0f)) continue;
        for (int i = threadIdx.x; i < NP; i += NT) acc[i] = 0;
        __syncthreads();
        bp_scatter<S0, S1, S2, NW, MERGE>(bj, q, v, ct, st, scale, acc, runs, ends);
        __syncthreads();
        const float inv = 1.0f / scale;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = threadIdx.x + NT * k;
            if (i < NP) sum[k] += (float)acc[i] * inv;
        }
        __syncthreads();
    }
    float *pad = bj.pads + (int64_t)bid * NPMAX;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x + NT * k;
        if (i >= NP) continue;
        const int z = i % P2, y = (i / P2) % P1, x = i / (P1 * P2);
        const int gx = q.B[0] + x, gy = q.B[1] + y, gz = q.B[2] + z;
        if (gx >= g.n[0] || gy >= g.n[1] || gz >= g.n[2]) continue;
        if (x < S0 && y < S1 && z < S2) bj.g_vol[((int64_t)gx * g.n[1] + gy) * g.n[2] + gz] = sum[k];
        else pad[i] = sum[k];
    }
}

// Waves per SIMD that the LDS of one workgroup (box + run staging) allows
// on a 160 KB CU, at most six: the register budget is set to match, so the
// compiler does not trade occupancy the LDS cannot use for registers.
constexpr int bwd_waves_per_simd(int L, int W, int H, int NW) {
    const int bytes = 4 * (L + 1) * (W + 1) * (H + 1) + NW * 64 * (int)(sizeof(RunP) + sizeof(int));
    const int wg = (160 * 1024) / bytes;
    const int w = wg * NW / 4;
    return w < 1 ? 1 : w > 6 ? 6 : w;
}

// L x W x H cells per brick (L along the axis the view's rays mostly
// follow), NW waves per workgroup.
template <int L, int W, int H, int NW, bool SUM, bool MERGE, int ZC>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(bwd_waves_per_simd(L, W, H, NW))))
void k_project_bwd(BwdTab t) {
    constexpr int NPMAX = (L + 1) * (W + 1) * (H + 1);
    __shared__ int acc[NPMAX];
    __shared__ RunP runs[NW][64];
    __shared__ int ends[NW][64];
    // within each scan, each XCD takes one contiguous range of its (view,
    // column chunk) items
    const int job = job_of(t, (int)blockIdx.x);
    const BwdK &bj = t.s[job];
    const int local = job_item(t, job, (int)blockIdx.x);
    if (local >= bj.items) return;
    if constexpr (SUM) {
        // summed over views: one orientation for all views (the first's)
        if (bj.orient[0])
            bp_summed<W, L, H, NW, NPMAX, MERGE>(bj, local, acc, runs, ends);
        else
            bp_summed<L, W, H, NW, NPMAX, MERGE>(bj, local, acc, runs, ends);
    } else {
        const int view = local / bj.nbv, item = local - view * bj.nbv;
        if (bj.orient[view])
            bp_column<W, L, H, NW, NPMAX, MERGE, ZC>(bj, view, item, acc, runs, ends);
        else
            bp_column<L, W, H, NW, NPMAX, MERGE, ZC>(bj, view, item, acc, runs, ends);
    }
}

// Fix-up of the brick faces: a voxel on the low face of its brick, where the
// brick below it on that axis staged its pad, gets the pads of the bricks
// below it, added in a fixed order (neighbour mask 1..7), and its share of
// vmax.  Axis-2 faces take part only at chunk boundaries (b2 a multiple of
// zc): inside a chunk the pad was carried.  The face voxels are walked by
// rows: family a holds the planes p_a = k S_a (k >= 1; family 2 only at chunk
// boundaries); a row is one line of such a plane along its faster axis, and a
// voxel that a lower family's plane also holds is left to that family, so
// each face voxel is completed once.  Blocks stride over one view's rows
// (one atomic for vmax per block).
template <int S0, int S1, int S2, int NPMAX>
__device__ __forceinline__ void bp_fixup(const BwdK &bj, int view, int sum_views, float *red) {
    constexpr int S[3] = {S0, S1, S2};
    constexpr int P1 = S1 + 1, P2 = S2 + 1;
    const GridK &g = bj.g;
    const int nb[3] = {(g.n[0] + S0 - 1) / S0, (g.n[1] + S1 - 1) / S1, (g.n[2] + S2 - 1) / S2};
    const int zc = sum_views ? 1 : bj.zc;
    const int nz = (nb[2] - 1) / zc;        // axis-2 planes at chunk boundaries
    // work rows: family 0 (axis-0 planes) and family 1 (axis-1 planes) are
    // lines along axis 2, rows_per lines to a row of work; family 2: per
    // (p0, p1) line along axis 2 its nz face voxels, taken by neighbouring
    // lanes, so a wave reads whole lines of memory (the face voxels are S2
    // floats apart)
    const int n2 = g.n[2];
    const int lpr = max(1, (int)blockDim.x / n2);                  // lines per row, families 0-1
    int zs = 1;
    while (zs < nz) zs <<= 1;
    const int lines2 = max(1, (int)blockDim.x / zs);               // lines per row, family 2
    const int l0 = (nb[0] - 1) * g.n[1], l1 = (nb[1] - 1) * g.n[0];  // lines of families 0, 1
    const int r0 = (l0 + lpr - 1) / lpr, r1 = (l1 + lpr - 1) / lpr;
    const int r2 = nz > 0 ? (g.n[0] * g.n[1] + lines2 - 1) / lines2 : 0;
    float *out = bj.g_vol + (sum_views ? 0 : (int64_t)view * bj.stride);
    const float *pads = bj.pads + (int64_t)view * bj.nbb * NPMAX;
    float mx = 0.0f;
    for (int row = blockIdx.x; row < r0 + r1 + r2; row += gridDim.x) {
      const int fam = row < r0 ? 0 : (row < r0 + r1 ? 1 : 2);
      const int span = fam < 2 ? lpr * n2 : lines2 * zs;       // entries of this row
      for (int e = threadIdx.x; e < span; e += blockDim.x) {
        int p[3];
        if (fam < 2) {
            const int line = (fam == 0 ? row : row - r0) * lpr + e / n2;
            if (line >= (fam == 0 ? l0 : l1)) continue;
            p[2] = e - (e / n2) * n2;
            if (fam == 0) {
                p[0] = (line / g.n[1] + 1) * S0;
                p[1] = line - (line / g.n[1]) * g.n[1];
            } else {
                p[1] = (line / g.n[0] + 1) * S1;
                p[0] = line - (line / g.n[0]) * g.n[0];
            }
        } else {
            const int k = e & (zs - 1), line = (row - r0 - r1) * lines2 + e / zs;
            if (k >= nz || line >= g.n[0] * g.n[1]) continue;
            p[0] = line / g.n[1];
            p[1] = line - p[0] * g.n[1];
            p[2] = (k + 1) * zc * S2;
        }
        if (p[0] >= g.n[0] || p[1] >= g.n[1] || p[2] >= g.n[2]) continue;
        int b[3], l[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            b[a] = p[a] / S[a];                 // constant divisors
            l[a] = p[a] - b[a] * S[a];
        }
        int mask = 0;
        if (l[0] == 0 && b[0] > 0) mask |= 1;
        if (l[1] == 0 && b[1] > 0) mask |= 2;
        if (l[2] == 0 && b[2] > 0 && b[2] % zc == 0) mask |= 4;
        if (!(mask >> fam & 1) || (mask & ((1 << fam) - 1))) continue;
        float sum = 0.0f;
#pragma unroll
        for (int d = 1; d < 8; ++d) {
            if ((d & mask) != d) continue;
            const int q0 = b[0] - (d & 1), q1 = b[1] - ((d >> 1) & 1), q2 = b[2] - ((d >> 2) & 1);
            const int lq0 = (d & 1) ? S0 : l[0], lq1 = (d & 2) ? S1 : l[1],
                      lq2 = (d & 4) ? S2 : l[2];
            const int nbid = (q0 * nb[1] + q1) * nb[2] + q2;
            sum += pads[(int64_t)nbid * NPMAX + (lq0 * P1 + lq1) * P2 + lq2];
        }
        float *o = out + ((int64_t)p[0] * g.n[1] + p[1]) * g.n[2] + p[2];
        const float val = *o + sum;
        *o = val;
        mx = fmaxf(mx, fabsf(val));
      }
    }
    if (bj.vmax && !sum_views) {
        mx = wave_max(mx);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
            if (mx > 0.0f) atomicMax(&bj.vmax[view], __float_as_uint(mx));
        }
    }
}

template <int L, int W, int H>
__global__ __launch_bounds__(256) void k_project_bwd_fixup(BwdK bj, int sum_views) {
    constexpr int NPMAX = (L + 1) * (W + 1) * (H + 1);
    __shared__ float red[4];
    const int view = blockIdx.y;
    if (bj.orient[view])
        bp_fixup<W, L, H, NPMAX>(bj, view, sum_views, red);
    else
        bp_fixup<L, W, H, NPMAX>(bj, view, sum_views, red);
}

// Geometry constants of the per-view bound on contributions per voxel
// (see k_project_bwd): largest magnification over the volume, the
// perspective spread per mm of depth, the volume's radius and half height.
static BoundK make_bound(const GridK &g, const ConeK &c) {
    BoundK b;
    double R = 0.0;
    for (int a = 0; a < 2; ++a) R += fmax(c.lo[a] * c.lo[a], c.hi[a] * c.hi[a]);
    R = sqrt(R);
    const double Z = fmax(fabs(c.lo[2]), fabs(c.hi[2]));
    // rounded up so the bound stays an upper bound in float
    b.mag = (float)(c.sdd / (c.sad - R) * (1.0 + 1e-6));
    b.persp = (float)(c.sdd / ((c.sad - R) * (c.sad - R)) * (1.0 + 1e-6));
    b.R = (float)(R * (1.0 + 1e-6));
    b.Z = (float)(Z * (1.0 + 1e-6));
    b.two_hx = (float)(2.0 * g.hd[0]);
    b.two_hy = (float)(2.0 * g.hd[1]);
    b.two_hz = (float)(2.0 * g.hd[2]);
    b.inv_du = (float)(1.0 / c.du * (1.0 + 1e-6));
    b.inv_dv = (float)(1.0 / c.dv * (1.0 + 1e-6));
    b.diag = (float)(2.0 * sqrt(g.hd[0] * g.hd[0] + g.hd[1] * g.hd[1] + g.hd[2] * g.hd[2]) *
                     (1.0 + 1e-6));
    return b;
}

template <int WU, int WV, int AU>
static void project_tiled(const ProjJob *jobs, int n, hipStream_t s) {
    constexpr int BU = WU * AU, BV = WV * (4 / AU);
    ProjTab t{};
    t.n = n;
    t.first[0] = 0;
    for (int k = 0; k < n; ++k) {
        const ProjJob &j = jobs[k];
        ProjK &p = t.s[k];
        p.vol = j.vol;
        p.stride = j.stride;
        p.g = j.g;
        p.c = j.c;
        p.mk = j.paired ? make_march_paired(j.g) : make_march(j.g);
        p.angles = j.angles;
        p.proj = j.proj;
        p.tiles_u = (j.c.nu + BU - 1) / BU;
        p.ntiles = p.tiles_u * ((j.c.nv + BV - 1) / BV);
        p.items = p.ntiles * j.V;
        t.first[k + 1] = t.first[k] + align8(p.items);
    }
    for (int k = n + 1; k <= MAXS; ++k) t.first[k] = t.first[n];
    if (t.first[n] == 0) return;
    if (jobs[0].paired)
        k_project<WU, WV, AU, true><<<(unsigned)t.first[n], 256, 0, s>>>(t);
    else
        k_project<WU, WV, AU, false><<<(unsigned)t.first[n], 256, 0, s>>>(t);
}

hipError_t launch_project_jobs(const ProjJob *jobs, int n, hipStream_t s) {
    if (n < 1 || n > MAXS) return hipErrorInvalidValue;
    for (int k = 1; k < n; ++k)
        if (jobs[k].paired != jobs[0].paired) return hipErrorInvalidValue;
    ProfScope prof_("project", s);
    switch (tune_get(KNOB_PROJECT_TILE)) {
        case 0: project_tiled<16, 4, 1>(jobs, n, s); break;
        case 1: project_tiled<8, 8, 2>(jobs, n, s); break;
        case 2: project_tiled<4, 16, 4>(jobs, n, s); break;
        case 3: project_tiled<2, 32, 4>(jobs, n, s); break;
        case 4: project_tiled<32, 2, 1>(jobs, n, s); break;
        case 5: project_tiled<1, 64, 4>(jobs, n, s); break;
        case 6: project_tiled<2, 32, 2>(jobs, n, s); break;
        case 7: project_tiled<1, 64, 2>(jobs, n, s); break;
        default: project_tiled<2, 32, 1>(jobs, n, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_project(const float *vol, int64_t stride, const GridK &g, const ConeK &c,
                          const float *angles, int V, float *proj, hipStream_t s) {
    const ProjJob j{vol, stride, g, c, angles, V, proj, false};
    return launch_project_jobs(&j, 1, s);
}

// Brick shapes of PMF_TUNE_BACKPROJECT_BRICK: L x W x H cells, waves.
struct BrickShape {
    int L, W, H, NW;
};
static const BrickShape kBricks[] = {{48, 16, 8, 8}, {48, 16, 8, 8}, {32, 16, 8, 8},
                                     {44, 16, 8, 8}, {44, 20, 8, 8}, {40, 20, 8, 8},
                                     {48, 16, 8, 8}, {64, 16, 8, 12}, {52, 16, 8, 8}};
constexpr int NBRICKS = sizeof(kBricks) / sizeof(kBricks[0]);

// Items per view: the brick count of the orientation with more bricks.
static int bricks_per_view(const GridK &g, int L, int W, int H) {
    auto cnt = [&](int s0, int s1) {
        return ((g.n[0] + s0 - 1) / s0) * ((g.n[1] + s1 - 1) / s1) * ((g.n[2] + H - 1) / H);
    };
    return std::max(cnt(L, W), cnt(W, L));
}

// Work items per view in per-view mode: (b0, b1) columns x chunks, for the
// orientation with more.
static int column_items_per_view(const GridK &g, int L, int W, int H, int zc) {
    const int nz = ((g.n[2] + H - 1) / H + zc - 1) / zc;
    auto cnt = [&](int s0, int s1) { return ((g.n[0] + s0 - 1) / s0) * ((g.n[1] + s1 - 1) / s1) * nz; };
    return std::max(cnt(L, W), cnt(W, L));
}

// Workspace: the per-ray table, two words of statistics and the orientation
// per view, then the pad boxes (sized for the largest brick shape, so the
// tuner can switch shapes on one workspace).
static size_t pad_floats(const GridK &g) {
    size_t m = 0;
    for (const BrickShape &b : kBricks)
        m = std::max(m, (size_t)bricks_per_view(g, b.L, b.W, b.H) * (size_t)(b.L + 1) *
                            (size_t)(b.W + 1) * (size_t)(b.H + 1));
    return m;
}

size_t project_bwd_workspace(const GridK &g, const pmf_cone_t &c, int V) {
    return align256(sizeof(RayK) * (size_t)c.nu * (size_t)c.nv * (size_t)V) +
           align256(sizeof(unsigned) * 2 * (size_t)V) + align256(sizeof(int) * (size_t)V) +
           align256(sizeof(float) * pad_floats(g) * (size_t)V);
}

template <int L, int W, int H, int NW, bool MERGE, int ZC>
static hipError_t project_bwd_bricks(const BwdJob *jobs, int n, hipStream_t s) {
    constexpr int NPMAX = (L + 1) * (W + 1) * (H + 1);
    const bool sum_views = jobs[0].stride == 0;
    BwdTab t{};
    t.n = n;
    t.first[0] = 0;
    for (int k = 0; k < n; ++k) {
        const BwdJob &j = jobs[k];
        if ((j.stride == 0) != sum_views) return hipErrorInvalidValue;
        char *w = (char *)j.ws;
        RayK *rays = (RayK *)w;
        w += align256(sizeof(RayK) * (size_t)j.c.nu * (size_t)j.c.nv * (size_t)j.V);
        unsigned *stats = (unsigned *)w;
        w += align256(sizeof(unsigned) * 2 * (size_t)j.V);
        int *orient = (int *)w;
        w += align256(sizeof(int) * (size_t)j.V);
        float *pads = (float *)w;
        // stats[2v] = 0 (max), stats[2v+1] = +inf (min)
        hipError_t e = launch_fill_pair_u32(stats, j.V, 0u, 0x7f800000u, s);
        if (e != hipSuccess) return e;
        {
            ProfScope prof_("ray_table", s);
            const int per_view = (j.c.nu * j.c.nv + 255) / 256;
            dim3 grid((unsigned)(per_view < 64 ? per_view : 64), (unsigned)j.V);
            k_ray_table<<<grid, 256, 0, s>>>(j.g, j.c, j.angles, j.g_proj, rays, stats, orient);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        BwdK &b = t.s[k];
        b.g_proj = j.g_proj;
        b.g = j.g;
        b.c = j.c;
        b.angles = j.angles;
        b.rays = rays;
        b.stats = stats;
        b.orient = orient;
        b.V = j.V;
        b.g_vol = j.g_vol;
        b.stride = j.stride;
        b.pads = pads;
        b.nbb = bricks_per_view(j.g, L, W, H);
        b.zc = sum_views ? 1 : ZC;
        b.nbv = sum_views ? b.nbb : column_items_per_view(j.g, L, W, H, b.zc);
        b.items = b.nbv * (sum_views ? 1 : j.V);
        b.kb = make_bound(j.g, j.c);
        b.mk = make_march(j.g);
        b.vmax = j.vmax;
        t.first[k + 1] = t.first[k] + align8(b.items);
    }
    for (int k = n + 1; k <= MAXS; ++k) t.first[k] = t.first[n];
    {
        ProfScope prof_("project_bwd", s);
        if (sum_views)
            k_project_bwd<L, W, H, NW, true, MERGE, 1><<<(unsigned)t.first[n], 64 * NW, 0, s>>>(t);
        else
            k_project_bwd<L, W, H, NW, false, MERGE, ZC><<<(unsigned)t.first[n], 64 * NW, 0, s>>>(t);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int k = 0; k < n; ++k) {
        const int64_t N = grid_size(t.s[k].g);
        ProfScope prof_("project_bwd_fixup", s);
        // blocks per view: about 16k over the views (measured: 2k, 4k, 8k
        // and 16k blocks took 0.235, 0.202, 0.185 and 0.178 ms at 32 views)
        const int V = sum_views ? 1 : t.s[k].V;
        const int per_view = std::max(1, std::min(2048, 16384 / V));
        (void)N;
        k_project_bwd_fixup<L, W, H><<<dim3((unsigned)per_view, (unsigned)V), 256, 0, s>>>(
            t.s[k], sum_views ? 1 : 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    (void)NPMAX;
    return hipSuccess;
}

// A chunked walk needs enough workgroups to fill the chip (a few per CU):
// a launch with few views (the plain schedule's one) takes shorter chunks,
// halving them until the column-chunk items reach 1536.
template <int L, int W, int H, int NW, bool MERGE, int ZC>
static hipError_t project_bwd_chunked(const BwdJob *jobs, int n, hipStream_t s) {
    if constexpr (ZC > 1) {
        int64_t items = 0;
        for (int k = 0; k < n; ++k) items += (int64_t)jobs[k].V * column_items_per_view(jobs[k].g, L, W, H, ZC);
        if (jobs[0].stride != 0 && items < 1536)
            return project_bwd_chunked<L, W, H, NW, MERGE, ZC / 2>(jobs, n, s);
    }
    return project_bwd_bricks<L, W, H, NW, MERGE, ZC>(jobs, n, s);
}

hipError_t launch_project_bwd_jobs(const BwdJob *jobs, int n, hipStream_t s) {
    if (n < 1 || n > MAXS) return hipErrorInvalidValue;
    static_assert(NBRICKS == 9, "tune candidates");
    switch (tune_get(KNOB_BACKPROJECT_BRICK)) {
        case 1: return project_bwd_bricks<48, 16, 8, 8, false, 1>(jobs, n, s);
        case 2: return project_bwd_chunked<32, 16, 8, 8, true, 8>(jobs, n, s);
        case 3: return project_bwd_chunked<44, 16, 8, 8, true, 8>(jobs, n, s);
        case 4: return project_bwd_chunked<44, 20, 8, 8, true, 8>(jobs, n, s);
        case 5: return project_bwd_chunked<40, 20, 8, 8, true, 8>(jobs, n, s);
        case 6: return project_bwd_chunked<48, 16, 8, 8, true, 8>(jobs, n, s);
        case 7: return project_bwd_chunked<64, 16, 8, 12, true, 8>(jobs, n, s);
        case 8: return project_bwd_chunked<52, 16, 8, 8, true, 8>(jobs, n, s);
        default: return project_bwd_bricks<48, 16, 8, 8, true, 1>(jobs, n, s);
    }
}

hipError_t launch_project_bwd(const float *g_proj, const GridK &g, const ConeK &c,
                              const float *angles, int V, float *g_vol, int64_t stride, void *ws,
                              hipStream_t s, unsigned *vmax) {
    const BwdJob j{g_proj, g, c, angles, V, g_vol, stride, ws, vmax};
    return launch_project_bwd_jobs(&j, 1, s);
}

}  // namespace pmf
