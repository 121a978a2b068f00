// common.hip -- grid/geometry descriptors and fill kernels.
#include <math.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "pmf_internal.h"

namespace pmf {

// ------------------------------------------------------------- profiling
static std::atomic<int> g_prof_on{0};
static std::mutex g_prof_mu;
static std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> g_prof;

ProfScope::ProfScope(const char *n, hipStream_t s) : name(n), stream(s), on(false) {
    if (!n || !g_prof_on.load(std::memory_order_relaxed)) return;   // no name: never recorded
    if (hipEventCreate(&start) != hipSuccess) return;
    if (hipEventCreate(&stop) != hipSuccess) {
        (void)hipEventDestroy(start);
        return;
    }
    on = hipEventRecord(start, stream) == hipSuccess;
    if (!on) {
        (void)hipEventDestroy(start);
        (void)hipEventDestroy(stop);
    }
}

ProfScope::~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(stop, stream);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[name].push_back({start, stop});
}

int profile_enable(int on) { return g_prof_on.exchange(on ? 1 : 0); }

// ------------------------------------------------------------- launch shapes
static const int g_tune_count[KNOB_COUNT] = {9, 9, 8};
static std::atomic<int> g_tune[KNOB_COUNT] = {{5}, {4}, {0}};

int tune_candidates(int knob) { return knob >= 0 && knob < KNOB_COUNT ? g_tune_count[knob] : 0; }

int tune_get(int knob) {
    return knob >= 0 && knob < KNOB_COUNT ? g_tune[knob].load(std::memory_order_relaxed) : 0;
}

int tune_set(int knob, int value) {
    if (knob < 0 || knob >= KNOB_COUNT || value < 0 || value >= g_tune_count[knob]) return -1;
    return g_tune[knob].exchange(value);
}

int profile_read(const char *name, double *total_ms, int64_t *count) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        auto it = g_prof.find(name);
        if (it != g_prof.end()) {
            ev.swap(it->second);
            g_prof.erase(it);
        }
    }
    double tot = 0.0;
    int rc = 0;
    for (auto &p : ev) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.second) != hipSuccess ||
            hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            rc = -1;
        tot += ms;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    *total_ms = tot;
    *count = (int64_t)ev.size();
    return rc;
}

size_t profile_names(char *buf, size_t len) {
    std::string all;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (auto &kv : g_prof) {
            if (!all.empty()) all += ",";
            all += kv.first;
        }
    }
    if (buf && len > 0) {
        size_t n = all.size() < len - 1 ? all.size() : len - 1;
        memcpy(buf, all.data(), n);
        buf[n] = 0;
    }
    return all.size();
}

GridK make_grid(const pmf_grid_t &g) {
    GridK k;
    for (int a = 0; a < 3; ++a) {
        k.n[a] = g.n[a];
        k.h[a] = g.h[a];
        k.hd[a] = (double)g.h[a];
        k.inv_h[a] = (float)(1.0 / (double)g.h[a]);
        k.c0d[a] = (double)g.center[a] - 0.5 * (double)(g.n[a] - 1) * (double)g.h[a];
        k.c0[a] = (float)k.c0d[a];
    }
    return k;
}

AxisMap make_axis_map(const GridK &out, const GridK &lvl) {
    AxisMap m;
    for (int a = 0; a < 3; ++a) {
        m.n[a] = lvl.n[a];
        bool same = out.n[a] == lvl.n[a] && out.hd[a] == lvl.hd[a] && out.c0d[a] == lvl.c0d[a];
        m.ident[a] = same ? 1 : 0;
        if (same) {
            m.scale[a] = 1.0f;
            m.off[a] = 0.0f;
        } else {
            m.scale[a] = (float)(out.hd[a] / lvl.hd[a]);
            m.off[a] = (float)((out.c0d[a] - lvl.c0d[a]) / lvl.hd[a]);
        }
    }
    return m;
}

ConeK make_cone(const pmf_cone_t &c, const GridK &g) {
    ConeK k;
    k.sad = c.sad;
    k.sdd = c.sdd;
    k.du = c.du;
    k.dv = c.dv;
    k.off_u = c.off_u;
    k.off_v = c.off_v;
    k.nu = c.nu;
    k.nv = c.nv;
    double step = c.step;
    if (!(step > 0.0)) step = 0.5 * fmin(fmin(g.hd[0], g.hd[1]), g.hd[2]);
    k.step = step;
    for (int a = 0; a < 3; ++a) {
        k.lo[a] = g.c0d[a] - 0.5 * g.hd[a];
        k.hi[a] = g.c0d[a] + ((double)g.n[a] - 0.5) * g.hd[a];
    }
    return k;
}

__global__ void k_fill(float *__restrict__ p, int64_t n, float v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_pair_u32(uint32_t *__restrict__ p, int64_t n, uint32_t a, uint32_t b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        p[2 * i] = a;
        p[2 * i + 1] = b;
    }
}

__global__ void k_accumulate(float *__restrict__ dst, const float *__restrict__ src, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] += src[i];
}

// out = max |x| over n floats, as the bits of a non-negative float (which
// order like unsigned integers); *out must hold 0 beforehand.
__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ x, int64_t n,
                                                uint32_t *__restrict__ out) {
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[i]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(out, __float_as_uint(m));
}

// out[0] = max of in[0..n) (float bits of non-negative floats), one block.
__global__ __launch_bounds__(256) void k_max_u32(const uint32_t *__restrict__ in, int n,
                                                 uint32_t *__restrict__ out) {
    __shared__ uint32_t red[4];
    uint32_t m = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = max(m, in[i]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// dst[i] = (float) fix[i] / fix_scale(*mx)  (+ dst[i] when add)
__global__ __launch_bounds__(256) void k_fix_to_float(const long long *__restrict__ fix, int64_t n,
                                                      const uint32_t *__restrict__ mx, int add,
                                                      float *__restrict__ dst) {
    const double sc = fix_scale(*mx);
    const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = (float)((double)fix[i] * inv);
        dst[i] = add ? dst[i] + v : v;
    }
}

static unsigned fill_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    {
        ProfScope prof_("fill", s);
        k_fill<<<fill_blocks(n), 256, 0, s>>>(p, n, v);
    }
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    {
        ProfScope prof_("fill", s);
        k_fill_i32<<<fill_blocks(n), 256, 0, s>>>(p, n, v);
    }
    return hipGetLastError();
}

hipError_t launch_fill_pair_u32(uint32_t *p, int64_t n, uint32_t a, uint32_t b, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    {
        ProfScope prof_("fill", s);
        k_fill_pair_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, a, b);
    }
    return hipGetLastError();
}

hipError_t launch_absmax(const float *x, int64_t n, uint32_t *out, hipStream_t s) {
    hipError_t e = launch_fill_i32((int32_t *)out, 1, 0, s);
    if (e != hipSuccess || n <= 0) return e;
    {
        ProfScope prof_("absmax", s);
        k_absmax<<<fill_blocks(n) < 1024 ? fill_blocks(n) : 1024, 256, 0, s>>>(x, n, out);
    }
    return hipGetLastError();
}

hipError_t launch_max_u32(const uint32_t *in, int n, uint32_t *out, hipStream_t s) {
    k_max_u32<<<1, 256, 0, s>>>(in, n, out);
    return hipGetLastError();
}

hipError_t launch_fix_to_float(const long long *fix, int64_t n, const uint32_t *mx, bool add,
                               float *dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    {
        ProfScope prof_("fix_to_float", s);
        k_fix_to_float<<<fill_blocks(n), 256, 0, s>>>(fix, n, mx, add ? 1 : 0, dst);
    }
    return hipGetLastError();
}

hipError_t launch_accumulate(float *dst, const float *src, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    {
        ProfScope prof_("accumulate", s);
        k_accumulate<<<fill_blocks(n), 256, 0, s>>>(dst, src, n);
    }
    return hipGetLastError();
}

}  // namespace pmf
