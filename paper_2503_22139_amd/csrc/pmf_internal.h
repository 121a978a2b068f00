// pmf_internal.h -- shared definitions of the gfx950 kernels and the C-ABI layer.
//
// Kernel-side descriptions of grids and cone-beam geometry, the trilinear
// stencil used by every step (warp, DVF upsampling, ray samples), the
// per-ray set-up of the midpoint-rule line integral, and the declarations of
// the host-side launchers implemented in the .hip files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmf.h"

namespace pmf {

// ----------------------------------------------------------------- grids
struct GridK {
    int n[3];
    float h[3];
    float inv_h[3];
    float c0[3];     // centre of voxel (0,0,0), float
    double c0d[3];   // same, double (ray set-up)
    double hd[3];
};

GridK make_grid(const pmf_grid_t &g);
__host__ __device__ inline int64_t grid_size(const GridK &g) { return (int64_t)g.n[0] * g.n[1] * g.n[2]; }

// Mapping of an output grid's voxel index onto a level grid's voxel units,
// u_a = off_a + i_a * scale_a (float fma), identity when the grids coincide.
struct AxisMap {
    float scale[3];
    float off[3];
    int n[3];       // level grid size
    int ident[3];   // 1 if the axis map is exactly the identity
};
AxisMap make_axis_map(const GridK &out, const GridK &lvl);

// ------------------------------------------------------------- geometry
struct ConeK {
    double sad, sdd, du, dv, off_u, off_v;
    double step;    // resolved step (mm)
    int nu, nv;
    double lo[3], hi[3];   // volume box
};
ConeK make_cone(const pmf_cone_t &c, const GridK &g);

// Per-ray constants of the midpoint rule, in voxel units of the grid:
// sample s sits at u = fma(s, su, bu) on each axis; n samples; step delta (mm).
struct alignas(16) RayK {
    float bu[3];
    float delta;
    float su[3];
    int n;
};

// --------------------------------------------------------- device helpers
#ifdef __HIPCC__
// 64-bit fixed point for scatters that cannot stay in LDS: with M the largest
// magnitude of any single contribution (bits of a non-negative float), each
// contribution x becomes llrint(x 2^40 / M), so it is exact to 2^-40 M and
// integer sums are independent of the order of the additions (results are
// bit-reproducible); a sum overflows only beyond 2^23 contributions of size
// M into one entry.
__host__ __device__ inline double fix_scale(uint32_t max_bits) {
    union {
        uint32_t u;
        float f;
    } c;
    c.u = max_bits;
    return c.f > 0.0f ? 1099511627776.0 / (double)c.f : 0.0;
}
__device__ __forceinline__ void fix_add(long long *dst, double x, double scale) {
    atomicAdd((unsigned long long *)dst, (unsigned long long)__double2ll_rn(x * scale));
}

// Trilinear coordinate on one axis: false if u is beyond the half-voxel rim
// (or NaN); otherwise the clamped cell index i in [0, n-2] and fraction f.
__device__ __forceinline__ bool axis_cell(float u, int n, int &i, float &f) {
    if (!(u >= -0.5f && u <= (float)n - 0.5f)) return false;
    float uc = fminf(fmaxf(u, 0.0f), (float)(n - 1));
    int ii = (int)floorf(uc);
    ii = ii < n - 2 ? ii : n - 2;
    i = ii;
    f = uc - (float)ii;
    return true;
}

// The same decision for the point idx + t on one axis (voxel units), idx a
// voxel index and t a displacement in voxels: the cell and fraction that
// axis_cell(idx + t) gives in exact arithmetic, decided from t alone.  The
// comparisons are exact (idx + 1/2 and n - 1 - idx are exact floats) and
// floor(t) is exact, so a point near a cell face takes the side its
// displacement puts it on; only t itself is rounded, at its own ulp rather
// than at the ulp of idx + t (up to 1.5e-5 voxel on a 256-voxel axis).
__device__ __forceinline__ bool disp_cell(int idx, float t, int n, int &i, float &f) {
    const float fi = (float)idx;
    if (!(t >= -0.5f - fi && t <= (float)n - 0.5f - fi)) return false;
    if (t <= -fi) {                     // on the rim below the first centre
        i = 0;
        f = 0.0f;
    } else if (t >= (float)(n - 1) - fi) {   // on the rim above the last centre
        i = n - 2;
        f = 1.0f;
    } else {
        const float fl = floorf(t);
        i = idx + (int)fl;
        f = t - fl;
    }
    return true;
}

// Derivative switch of disp_cell's point: strictly inside the voxel-centre hull.
__device__ __forceinline__ float disp_free(int idx, float t, int n) {
    const float fi = (float)idx;
    return (t > -fi && t < (float)(n - 1) - fi) ? 1.0f : 0.0f;
}

__device__ __forceinline__ float lerp1(float a, float b, float t) { return fmaf(t, b - a, a); }

// Trilinear read at voxel-unit coordinate (u0,u1,u2); 0 outside the box.
__device__ __forceinline__ float sample_u(const float *__restrict__ vol, const int n[3], float u0,
                                          float u1, float u2) {
    int i0, i1, i2;
    float f0, f1, f2;
    if (!axis_cell(u0, n[0], i0, f0) || !axis_cell(u1, n[1], i1, f1) ||
        !axis_cell(u2, n[2], i2, f2))
        return 0.0f;
    const int s1 = n[2], s0 = n[1] * n[2];
    const float *p = vol + ((i0 * n[1] + i1) * n[2] + i2);
    float c00 = lerp1(p[0], p[1], f2);
    float c01 = lerp1(p[s1], p[s1 + 1], f2);
    float c10 = lerp1(p[s0], p[s0 + 1], f2);
    float c11 = lerp1(p[s0 + s1], p[s0 + s1 + 1], f2);
    return lerp1(lerp1(c00, c01, f1), lerp1(c10, c11, f1), f0);
}

// Trilinear read at the point (i0 + t0, i1 + t1, i2 + t2): voxel indices
// plus displacements in voxels (see disp_cell); 0 outside the box.
__device__ __forceinline__ float sample_disp(const float *__restrict__ vol, const int n[3], int i0,
                                             int i1, int i2, float t0, float t1, float t2) {
    int c0, c1, c2;
    float f0, f1, f2;
    if (!disp_cell(i0, t0, n[0], c0, f0) || !disp_cell(i1, t1, n[1], c1, f1) ||
        !disp_cell(i2, t2, n[2], c2, f2))
        return 0.0f;
    const int s1 = n[2], s0 = n[1] * n[2];
    const float *p = vol + ((c0 * n[1] + c1) * n[2] + c2);
    float c00 = lerp1(p[0], p[1], f2);
    float c01 = lerp1(p[s1], p[s1 + 1], f2);
    float c10 = lerp1(p[s0], p[s0 + 1], f2);
    float c11 = lerp1(p[s0 + s1], p[s0 + s1 + 1], f2);
    return lerp1(lerp1(c00, c01, f1), lerp1(c10, c11, f1), f0);
}

// Largest value over the 64 lanes (every lane receives it).
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float warp_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 64 lanes of a wave with DPP moves (VALU only, no LDS).
// The total is valid in lane 63 (other lanes hold partial sums).
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK,
                                                      BANK_MASK, true));
}
__device__ __forceinline__ float wave_sum_lane63(float v) {
    v += dpp_mov<0xB1>(v);              // quad_perm [1,0,3,2]: pairs
    v += dpp_mov<0x4E>(v);              // quad_perm [2,3,0,1]: quads
    v += dpp_mov<0x141>(v);             // row_half_mirror: 8 lanes
    v += dpp_mov<0x140>(v);             // row_mirror: 16 lanes (a row)
    v += dpp_mov<0x142, 0xa>(v);        // row_bcast:15 into rows 1, 3
    v += dpp_mov<0x143, 0xc>(v);        // row_bcast:31 into rows 2, 3
    return v;
}

// Sum of n partials by one full wave in a fixed order (lane i adds i, i + 64,
// ... in turn, then the wave's tree); the total is in lane 63.
__device__ __forceinline__ float wave_sum_partials(const float *__restrict__ p, int n) {
    float s = 0.0f;
#pragma unroll 8
    for (int i = (int)(threadIdx.x & 63); i < n; i += 64) s += p[i];
    return wave_sum_lane63(s);
}

// Orders the LDS accesses of one wavefront (a compiler barrier: the hardware
// performs a wavefront's LDS operations in order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, true);
}

// Inclusive prefix sum over the 64 lanes (lanes shifted in from outside a
// row read 0).
__device__ __forceinline__ int wave_incl_sum(int x) {
    x += dpp_i<0x111>(x);          // row_shr:1
    x += dpp_i<0x112>(x);          // row_shr:2
    x += dpp_i<0x114>(x);          // row_shr:4
    x += dpp_i<0x118>(x);          // row_shr:8
    x += dpp_i<0x142, 0xa>(x);     // row_bcast:15 into rows 1, 3
    x += dpp_i<0x143, 0xc>(x);     // row_bcast:31 into rows 2, 3
    return x;
}

// The permlane swaps exchange data between two registers across lanes
// 32 apart (swap32: a' = a's lanes 0-31 then b's lanes 0-31, b' = a's lanes
// 32-63 then b's lanes 32-63) or rows of 16 lanes (swap16: a' = rows a0 b0
// a2 b2, b' = rows a1 b1 a3 b3); a' + b' then sums lane L with lane L ^ 32
// (or L ^ 16) for a different value in each half (or row), in two
// instructions and without a lane select.
__device__ __forceinline__ void swap32(float &a, float &b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float &a, float &b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                    false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// Reduce-scatter of 32 per-lane values over the 64 lanes of a wave: returns
// the total over all lanes of value 16*b3 + 8*b2 + 4*b1 + 2*b0 + b4 (b_k =
// bit k of the lane; the same total in lanes L and L+32).  Each step pairs
// lanes that hold the same set of partial sums, keeps half of the set and
// adds the partner's copy of that half: 16 + 8 + 4 + 2 + 1 + 1 additions
// instead of 32 separate six-step reductions.  (A form that pairs halves and
// rows with the permlane swaps first, as the 16-value version below does,
// measured 7% slower in the rasterizer's adjoint, its one user.)
__device__ __forceinline__ float wave_reduce_scatter32(const float (&x)[32], int lane) {
    const bool h3 = lane & 8, h2 = lane & 4, h1 = lane & 2, h0 = lane & 1, h4 = lane & 16;
    float a[16], b[8], c[4], d[2];
#pragma unroll
    for (int j = 0; j < 16; ++j) {     // partner: row_mirror (lane ^ 15 within 16)
        const float keep = h3 ? x[16 + j] : x[j], send = h3 ? x[j] : x[16 + j];
        a[j] = keep + dpp_mov<0x140>(send);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {      // partner: row_half_mirror (lane ^ 7 within 8)
        const float keep = h2 ? a[8 + j] : a[j], send = h2 ? a[j] : a[8 + j];
        b[j] = keep + dpp_mov<0x141>(send);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {      // partner: lane ^ 2
        const float keep = h1 ? b[4 + j] : b[j], send = h1 ? b[j] : b[4 + j];
        c[j] = keep + dpp_mov<0x4E>(send);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {      // partner: lane ^ 1
        const float keep = h0 ? c[2 + j] : c[j], send = h0 ? c[j] : c[2 + j];
        d[j] = keep + dpp_mov<0xB1>(send);
    }
    const float keep = h4 ? d[1] : d[0], send = h4 ? d[0] : d[1];
    const float e = keep + __shfl_xor(send, 16, 64);
    return e + __shfl_xor(e, 32, 64);
}

__device__ __forceinline__ int scatter32_index(int lane) {
    return 16 * ((lane >> 3) & 1) + 8 * ((lane >> 2) & 1) + 4 * ((lane >> 1) & 1) +
           2 * (lane & 1) + ((lane >> 4) & 1);
}

// Reduce-scatter of 16 per-lane values over the 64 lanes of a wave: lane L
// returns the total over all lanes of value L >> 2 (lanes L .. L ^ 3 hold the
// same total).  Each step pairs lanes that hold the same set of partial sums,
// keeps half of the set and adds the partner's copy of that half; the halves
// and rows are paired by the permlane swaps (two instructions per pair, no
// lane select, no LDS permute), the lanes of a row by DPP.
__device__ __forceinline__ float wave_reduce_scatter16(const float (&x)[16], int lane) {
    const bool h3 = lane & 8, h2 = lane & 4;
    float a[8], b[4], c[2];
#pragma unroll
    for (int j = 0; j < 8; ++j) {      // value j + 8 b5
        float p = x[j], q = x[8 + j];
        swap32(p, q);
        a[j] = p + q;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {      // value j + 4 b4 + 8 b5
        float p = a[j], q = a[4 + j];
        swap16(p, q);
        b[j] = p + q;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {      // partner: row_mirror
        const float keep = h3 ? b[2 + j] : b[j], send = h3 ? b[j] : b[2 + j];
        c[j] = keep + dpp_mov<0x140>(send);
    }
    const float keep = h2 ? c[1] : c[0], send = h2 ? c[0] : c[1];
    float e = keep + dpp_mov<0x141>(send);          // partner: row_half_mirror
    e += dpp_mov<0x4E>(e);                          // lane ^ 2
    return e + dpp_mov<0xB1>(e);                    // lane ^ 1
}

__device__ __forceinline__ int scatter16_index(int lane) { return lane >> 2; }
#endif

// ------------------------------------------------------ ragged launches
// A ragged batch launches one kernel per stage for up to MAXS scans; a table
// in the kernel arguments gives each scan's parameters and its first
// workgroup.
constexpr int MAXS = 4;
#ifdef __HIPCC__
// Workgroup b of a G-workgroup launch runs on XCD b % 8 (the dispatcher deals
// workgroups round-robin over the 8 XCDs, each with its own L2).  The
// returned index gives each XCD one contiguous range of work items, so items
// that share cache lines (neighbouring bricks or tiles) share an L2.
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int k = b & 7, q = G >> 3, r = G & 7;
    return k * q + (k < r ? k : r) + (b >> 3);
}

// Item handled by workgroup b of table entry `job`.  Each entry's workgroup
// range starts at a multiple of 8 and has a multiple-of-8 length, so within
// it the XCD of a workgroup is (b - first) % 8 and xcd_block gives every XCD
// an equal, contiguous share of the entry's items; items past the entry's
// count (the padding) are left to the caller to skip.
template <class Tab>
__device__ __forceinline__ int job_item(const Tab &t, int job, int b) {
    return xcd_block(b - t.first[job], t.first[job + 1] - t.first[job]);
}

// index of the table entry that owns workgroup b (first[] is non-decreasing)
template <class Tab>
__device__ __forceinline__ int job_of(const Tab &t, int b) {
    int k = 0;
#pragma unroll
    for (int j = 1; j < MAXS; ++j) k += (j < t.n && b >= t.first[j]) ? 1 : 0;
    return k;
}
#endif

// ------------------------------------------------- basis upsampling helpers
constexpr int MAXL = 4, MAXB = 4;
struct LevelsK {
    const float *E[MAXL];
    AxisMap map[MAXL];
    int L, B;
};

#ifdef __HIPCC__
struct LevelStencil {
    int base;
    float f0, f1, f2;
    int s0, s1;  // strides of axes 0 and 1 in the level grid
    bool in;
};

__device__ __forceinline__ float level_coord(const AxisMap &m, int a, int i) {
    return m.ident[a] ? (float)i : fmaf((float)i, m.scale[a], m.off[a]);
}

__device__ __forceinline__ LevelStencil level_stencil(const AxisMap &m, int ix, int iy, int iz) {
    LevelStencil st;
    int i0, i1, i2;
    st.in = axis_cell(level_coord(m, 0, ix), m.n[0], i0, st.f0) &&
            axis_cell(level_coord(m, 1, iy), m.n[1], i1, st.f1) &&
            axis_cell(level_coord(m, 2, iz), m.n[2], i2, st.f2);
    st.s1 = m.n[2];
    st.s0 = m.n[1] * m.n[2];
    st.base = st.in ? (i0 * m.n[1] + i1) * m.n[2] + i2 : 0;
    return st;
}

__device__ __forceinline__ float stencil_read(const float *__restrict__ E, const LevelStencil &st) {
    const float *p = E + st.base;
    // on a voxel centre of the level grid (every interior voxel of a level
    // that shares the output grid) each lerp returns its first argument
    // exactly (fma(0, b - a, a) = a): one read instead of eight
    if (st.f0 == 0.0f && st.f1 == 0.0f && st.f2 == 0.0f) return p[0];
    const int s0 = st.s0, s1 = st.s1;
    float c00 = lerp1(p[0], p[1], st.f2);
    float c01 = lerp1(p[s1], p[s1 + 1], st.f2);
    float c10 = lerp1(p[s0], p[s0 + 1], st.f2);
    float c11 = lerp1(p[s0 + s1], p[s0 + s1 + 1], st.f2);
    return lerp1(lerp1(c00, c01, st.f1), lerp1(c10, c11, st.f1), st.f0);
}

// sv[l][b][k] = S(E_l[b*3+k], x_j) for the voxel (ix,iy,iz) of the output grid.
template <int L, int B>
__device__ __forceinline__ void basis_samples(const LevelsK &lv, int ix, int iy, int iz,
                                              float sv[L][B][3]) {
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const LevelStencil st = level_stencil(lv.map[l], ix, iy, iz);
        const int64_t Nl = (int64_t)lv.map[l].n[0] * lv.map[l].n[1] * lv.map[l].n[2];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                sv[l][b][k] = st.in ? stencil_read(lv.E[l] + (b * 3 + k) * Nl, st) : 0.0f;
    }
}
#endif

// Calls f(IC<L>{}, IC<B>{}) with compile-time level and basis counts.
template <int V>
struct IC {
    static constexpr int value = V;
};
template <typename F>
hipError_t dispatch_lb(int L, int B, F &&f) {
#define PMF_LB(l, b) \
    if (L == l && B == b) return f(IC<l>{}, IC<b>{});
    PMF_LB(1, 1) PMF_LB(1, 2) PMF_LB(1, 3) PMF_LB(1, 4)
    PMF_LB(2, 1) PMF_LB(2, 2) PMF_LB(2, 3) PMF_LB(2, 4)
    PMF_LB(3, 1) PMF_LB(3, 2) PMF_LB(3, 3) PMF_LB(3, 4)
    PMF_LB(4, 1) PMF_LB(4, 2) PMF_LB(4, 3) PMF_LB(4, 4)
#undef PMF_LB
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------- profiling
// When enabled (pmf_profile), each kernel launch is bracketed by two HIP
// events recorded on its stream; pmf_profile_read sums their elapsed times.
struct ProfScope {
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
    const char *name;
    hipStream_t stream;
    hipEvent_t start, stop;
    bool on;
};

int profile_enable(int on);
int profile_read(const char *name, double *total_ms, int64_t *count);
size_t profile_names(char *buf, size_t len);

// ------------------------------------------------------------- launch shapes
// Process-wide choice of launch shape per tunable kernel (index into that
// kernel's candidate list); set by pmf_tune_set or the autotuner.
enum Knob {
    KNOB_PROJECT_TILE = 0,
    KNOB_BACKPROJECT_BRICK = 1,
    KNOB_VOXELIZE_BWD = 2,
    KNOB_COUNT = 3
};
int tune_get(int knob);
int tune_set(int knob, int value);   // returns the previous value, or -1 if out of range
int tune_candidates(int knob);

// ------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.  Arguments were validated.
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// p[2i] = a, p[2i+1] = b for i < n
hipError_t launch_fill_pair_u32(uint32_t *p, int64_t n, uint32_t a, uint32_t b, hipStream_t s);
hipError_t launch_accumulate(float *dst, const float *src, int64_t n, hipStream_t s);
// *out = bits of max |x[i]| over n floats (out is cleared first)
hipError_t launch_absmax(const float *x, int64_t n, uint32_t *out, hipStream_t s);
// out[0] = max of n unsigned words (float bits of non-negative floats)
hipError_t launch_max_u32(const uint32_t *in, int n, uint32_t *out, hipStream_t s);
// dst = fix / fix_scale(*mx) (add: dst += ...)
hipError_t launch_fix_to_float(const long long *fix, int64_t n, const uint32_t *mx, bool add,
                               float *dst, hipStream_t s);

// voxelize
struct VoxPlan {
    int T[3];          // tile dims (voxels)
    int nt[3];         // tiles per axis
    int64_t ntiles;
    int64_t cap;       // capacity of the (tile, gaussian) list
    int maxtiles;      // Gaussians overlapping more tiles go to the large list
};
VoxPlan vox_plan(int64_t m, int c, const GridK &g);
size_t vox_workspace(const VoxPlan &p, int64_t m);
hipError_t launch_voxelize(const pmf_gauss_t &gs, const GridK &g, float k, float *vol,
                           const VoxPlan &p, void *ws, hipStream_t s);
hipError_t launch_voxelize_bwd(const pmf_gauss_t &gs, const GridK &g, float k, const float *g_vol,
                               const pmf_gauss_grad_t &gr, hipStream_t s);

// combine
hipError_t launch_combine(const LevelsK &lv, const float *coeff, int V, const GridK &out, float *dvf,
                          hipStream_t s);
size_t combine_bwd_workspace(const LevelsK &lv, const GridK *lvl_grids, int V, const GridK &out);
hipError_t launch_combine_bwd(const LevelsK &lv, const GridK *lvl_grids, const float *coeff, int V,
                              const GridK &out, const float *g_dvf, float *const *g_bases,
                              float *g_coeff, void *ws, hipStream_t s);
// separable transpose of the upsampling of one level, from a full-grid
// per-channel source G [C][N] (or from g_dvf/coeff when G is null)
hipError_t launch_upsample_adjoint(const LevelsK &lv, int l, const GridK &lvl_grid,
                                   const float *coeff, int V, const GridK &out, const float *g_dvf,
                                   const float *G, float *g_base, void *ws, hipStream_t s);
size_t upsample_adjoint_workspace(int C, const GridK &lvl_grid, const GridK &out, const AxisMap &m);

// warp
hipError_t launch_warp(const float *ref, const GridK &g, const float *dvf, int V, float *out,
                       hipStream_t s);
size_t warp_bwd_workspace(const GridK &g);
hipError_t launch_warp_bwd(const float *ref, const GridK &g, const float *dvf, int V,
                           const float *g_out, float *g_ref, float *g_dvf, void *ws,
                           hipStream_t s);

// projection
struct ProjJob {            // one scan's forward projection
    const float *vol;
    int64_t stride;         // elements between views' volumes (0: one volume)
    GridK g;
    ConeK c;
    const float *angles;
    int V;
    float *proj;
    bool paired;            // vol in the y-paired layout (2 floats per voxel; all jobs alike)
};
hipError_t launch_project_jobs(const ProjJob *jobs, int n, hipStream_t s);
hipError_t launch_project(const float *vol, int64_t stride, const GridK &g, const ConeK &c,
                          const float *angles, int V, float *proj, hipStream_t s);
struct BwdJob {             // one scan's back-projection (all jobs per view, or all summed)
    const float *g_proj;
    GridK g;
    ConeK c;
    const float *angles;
    int V;
    float *g_vol;
    int64_t stride;         // 0: sum over views into one volume
    void *ws;               // project_bwd_workspace(g, c, V) bytes
    unsigned *vmax;         // optional [V], zeroed: largest |g_vol| per view (float bits)
};
hipError_t launch_project_bwd_jobs(const BwdJob *jobs, int n, hipStream_t s);
size_t project_bwd_workspace(const GridK &g, const pmf_cone_t &c, int V);
// vmax (optional, [V] zeroed uint): largest |g_vol| of each view, as float bits
hipError_t launch_project_bwd(const float *g_proj, const GridK &g, const ConeK &c,
                              const float *angles, int V, float *g_vol, int64_t stride, void *ws,
                              hipStream_t s, unsigned *vmax = nullptr);

// loss
size_t fdk_workspace(const pmf_cone_t &c, int V);
hipError_t launch_fdk(const float *proj, const pmf_cone_t &c, const float *angles, int V,
                      const GridK &g, float *vol, void *ws, hipStream_t s);
hipError_t launch_grid_init(const float *vol, const GridK &g, const int m[3], float s,
                            float *mean, float *scale, float *quat, float *value, hipStream_t st);
size_t rasterize_workspace(int64_t m, const pmf_cone_t &c, int V);
hipError_t launch_rasterize(const pmf_gauss_t &gs, const pmf_cone_t &c, const float *angles,
                            int V, float k, float *proj, void *ws, hipStream_t s);
hipError_t launch_rasterize_bwd(const pmf_gauss_t &gs, const pmf_cone_t &c, const float *angles,
                                int V, float k, const float *g_proj, const pmf_gauss_grad_t &gg,
                                void *ws, hipStream_t s, bool rebin = true);
size_t l1_dssim_workspace(int nu, int nv, int V);
hipError_t launch_l1_dssim(const float *proj, const float *target, int nu, int nv, int V,
                           float lam, float *loss, float *g, void *ws, hipStream_t s);
size_t tv_workspace(int D);
hipError_t launch_tv(const float *vol, const GridK &g, const int corner[3], int D, float weight,
                     float *loss, float *g_vol, void *ws, hipStream_t s);
// pmf_tv_loss without a workspace: the partial sums live in a static device
// array sized for D <= TV_NOALLOC_MAX_D (hipErrorInvalidValue beyond).
constexpr int TV_NOALLOC_MAX_D = PMF_TV_NOALLOC_MAX_D;
hipError_t launch_tv_noalloc(const float *vol, const GridK &g, const int corner[3], int D,
                             float weight, float *loss, float *g_vol, hipStream_t s);
size_t normality_workspace(int L, int C);
hipError_t launch_normality(int L, int C, const float *const *bases, const GridK *lg,
                            float weight, float *loss, float *const *g, void *ws, hipStream_t s);
size_t l2_workspace(int64_t npix, int V);
hipError_t launch_l2(const float *proj, const float *target, int64_t npix, int V, float *loss,
                     float *g, void *ws, hipStream_t s);

// fused motion path
struct WPJob {              // one scan's forward: ws = warp_project_workspace bytes
    const float *ref;
    GridK g;
    LevelsK lv;
    const float *coeff;
    int V;
    ConeK c;
    const float *angles;
    float *proj;
    void *ws;
};
struct WPBJob {             // one scan's adjoint: ws = warp_project_bwd_workspace bytes
    const float *ref;
    GridK g;
    LevelsK lv;
    GridK lvl_grids[MAXL];
    const float *coeff;
    int V;
    ConeK c;
    const float *angles;
    const float *g_proj;
    float *g_ref;
    float *g_bases[MAXL];
    float *g_coeff;
    void *ws;
};
// All jobs share L and B.
hipError_t launch_warp_project_jobs(const WPJob *jobs, int n, hipStream_t s);
hipError_t launch_warp_project_bwd_jobs(const WPBJob *jobs, int n, hipStream_t s);
size_t warp_project_workspace(const LevelsK &lv, int V, const GridK &g, const pmf_cone_t &c);
hipError_t launch_warp_project(const float *ref, const GridK &g, const LevelsK &lv,
                               const float *coeff, int V, const ConeK &c, const float *angles,
                               float *proj, void *ws, hipStream_t s);
size_t warp_project_bwd_workspace(const LevelsK &lv, const GridK *lvl_grids, int V, const GridK &g,
                                  const pmf_cone_t &c);
hipError_t launch_warp_project_bwd(const float *ref, const GridK &g, const LevelsK &lv,
                                   const GridK *lvl_grids, const float *coeff, int V,
                                   const ConeK &c, const float *angles, const float *g_proj,
                                   float *g_ref, float *const *g_bases, float *g_coeff, void *ws,
                                   hipStream_t s);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int align8(int x) { return (x + 7) & ~7; }

}  // namespace pmf
