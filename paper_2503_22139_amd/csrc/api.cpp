// api.cpp -- the extern "C" entry points of libpmf.so (declared in pmf.h).
//
// Every entry point validates its arguments on the host before touching the
// HIP runtime, so a rejected call enqueues nothing.  Errors are reported as a
// pmf_status with a thread-local message.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string.h>

#include <string>
#include <vector>

#include <cmath>

#include "pmf_internal.h"

using namespace pmf;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return PMF_OK;
}

int hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return ok();
    return fail(PMF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(float x) { return isfinite(x) && x > 0.0f; }

int check_grid(const pmf_grid_t *g, const char *name) {
    if (!g) return fail(PMF_EINVAL, "%s: null grid", name);
    int64_t N = 1;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 2) return fail(PMF_EINVAL, "%s: n[%d] = %d < 2", name, a, g->n[a]);
        if (!finite_pos(g->h[a])) return fail(PMF_EINVAL, "%s: h[%d] must be > 0", name, a);
        if (!isfinite(g->center[a])) return fail(PMF_EINVAL, "%s: center not finite", name);
        N *= g->n[a];
    }
    if (N >= ((int64_t)1 << 31)) return fail(PMF_EINVAL, "%s: more than 2^31 voxels", name);
    return PMF_OK;
}

int check_march_grid(const pmf_grid_t *g);

int check_cone(const pmf_cone_t *c, const pmf_grid_t *g) {
    if (!c) return fail(PMF_EINVAL, "cone: null");
    if (!(isfinite(c->sad) && isfinite(c->sdd) && c->sad > 0.0f && c->sdd > c->sad))
        return fail(PMF_EINVAL, "cone: need 0 < SAD < SDD");
    if (c->nu < 1 || c->nv < 1) return fail(PMF_EINVAL, "cone: nu, nv must be >= 1");
    if ((int64_t)c->nu * c->nv >= ((int64_t)1 << 31))
        return fail(PMF_EINVAL, "cone: too many pixels");
    if (!finite_pos(c->du) || !finite_pos(c->dv)) return fail(PMF_EINVAL, "cone: du, dv must be > 0");
    if (!isfinite(c->off_u) || !isfinite(c->off_v) || !isfinite(c->step))
        return fail(PMF_EINVAL, "cone: offsets and step must be finite");
    // the volume box must lie strictly inside the source circle
    double rmax = 0.0;
    for (int q = 0; q < 4; ++q) {
        double x = g->center[0] + ((q & 1) ? 0.5 : -0.5) * g->n[0] * (double)g->h[0];
        double y = g->center[1] + ((q & 2) ? 0.5 : -0.5) * g->n[1] * (double)g->h[1];
        rmax = fmax(rmax, sqrt(x * x + y * y));
    }
    if (!(rmax < c->sad)) return fail(PMF_EINVAL, "cone: volume box reaches the source circle");
    return check_march_grid(g);
}

// The ray-march kernels index with 24-bit multiplies and 32-bit byte offsets.
int check_march_grid(const pmf_grid_t *g) {
    if ((int64_t)g->n[1] * g->n[2] >= ((int64_t)1 << 24))
        return fail(PMF_EUNSUPPORTED, "projection: n1*n2 must be < 2^24");
    if ((int64_t)g->n[0] * g->n[1] * g->n[2] >= ((int64_t)1 << 30))
        return fail(PMF_EUNSUPPORTED, "projection: more than 2^30 voxels");
    return PMF_OK;
}

int check_gauss(const pmf_gauss_t *gs) {
    if (!gs) return fail(PMF_EINVAL, "gaussians: null");
    if (gs->m < 0) return fail(PMF_EINVAL, "gaussians: m < 0");
    if (gs->c < 1) return fail(PMF_EINVAL, "gaussians: c must be >= 1");
    if (gs->c > 16) return fail(PMF_EUNSUPPORTED, "gaussians: c = %d > 16", gs->c);
    if (gs->m > ((int64_t)1 << 26)) return fail(PMF_EUNSUPPORTED, "gaussians: m > 2^26");
    if (gs->m > 0 && (!gs->mean || !gs->scale || !gs->quat || !gs->value))
        return fail(PMF_EINVAL, "gaussians: null array");
    return PMF_OK;
}

int check_k(float k) {
    if (!(k > 0.0f)) return fail(PMF_EINVAL, "trunc_k must be > 0 (or INFINITY)");
    return PMF_OK;
}

int check_ws(void *ws, size_t have, size_t need) {
    if (need == 0) return PMF_OK;
    if (!ws) return fail(PMF_EWORKSPACE, "workspace: null (need %zu bytes)", need);
    if (have < need) return fail(PMF_EWORKSPACE, "workspace: %zu bytes < %zu needed", have, need);
    return PMF_OK;
}

int check_levels(int L, int B, const float *const *bases, const pmf_grid_t *lvl, const char *what) {
    if (L < 1 || B < 1) return fail(PMF_EINVAL, "%s: L and B must be >= 1", what);
    if (L > MAXL || B > MAXB) return fail(PMF_EUNSUPPORTED, "%s: L <= 4 and B <= 4", what);
    if (!bases || !lvl) return fail(PMF_EINVAL, "%s: null level arrays", what);
    for (int l = 0; l < L; ++l) {
        if (!bases[l]) return fail(PMF_EINVAL, "%s: null basis pointer %d", what, l);
        int r = check_grid(&lvl[l], "level grid");
        if (r) return r;
    }
    return PMF_OK;
}

LevelsK make_levels(int L, int B, const float *const *bases, const pmf_grid_t *lvl,
                    const GridK &out, GridK *lg) {
    LevelsK lv;
    lv.L = L;
    lv.B = B;
    for (int l = 0; l < MAXL; ++l) {
        lv.E[l] = l < L ? bases[l] : nullptr;
        if (l < L) {
            lg[l] = make_grid(lvl[l]);
            lv.map[l] = make_axis_map(out, lg[l]);
        }
    }
    return lv;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

}  // namespace

#define PMF_CHECK(expr)         \
    do {                        \
        int r_ = (expr);        \
        if (r_ != PMF_OK) return r_; \
    } while (0)

// ------------------------------------------- autotuner with a shape cache
namespace {
// Cache key: the device (architecture, name, compute units) and every input
// of the projection's cost (grid, geometry, views).
std::string autotune_key(const pmf_grid_t *g, const pmf_cone_t *c, int V) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string dname = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        dname = std::string(prop.gcnArchName) + "/" + prop.name + "/" +
                std::to_string(prop.multiProcessorCount);
    for (char &ch : dname)
        if (ch == '\t' || ch == '\n' || ch == ' ') ch = '_';
    char buf[512];
    snprintf(buf, sizeof buf,
             "%s n=%d,%d,%d h=%.9g,%.9g,%.9g cone=%d,%d,%.9g,%.9g,%.9g,%.9g,%.9g,%.9g,%.9g V=%d",
             dname.c_str(), g->n[0], g->n[1], g->n[2], (double)g->h[0], (double)g->h[1],
             (double)g->h[2], c->nu, c->nv, (double)c->du, (double)c->dv, (double)c->sad,
             (double)c->sdd, (double)c->off_u, (double)c->off_v, (double)c->step, V);
    return buf;
}

// The last entry for key in the cache file: "key\ttile\tbrick" lines.
bool autotune_lookup(const char *path, const std::string &key, int &tile, int &brick) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    while (fgets(line, sizeof line, f)) {
        char *t1 = strchr(line, '\t');
        if (!t1) continue;
        *t1 = '\0';
        if (key != line) continue;
        int a = -1, b = -1;
        if (sscanf(t1 + 1, "%d\t%d", &a, &b) == 2 && a >= 0 &&
            a < tune_candidates(KNOB_PROJECT_TILE) && b >= 0 &&
            b < tune_candidates(KNOB_BACKPROJECT_BRICK)) {
            tile = a;
            brick = b;
            found = true;
        }
    }
    fclose(f);
    return found;
}
}  // namespace

extern "C" {

int pmf_version(void) { return PMF_VERSION; }

const char *pmf_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- voxelize
size_t pmf_voxelize_workspace(int64_t m, int32_t c, const pmf_grid_t *grid) {
    if (!grid || m < 0 || c < 1) return 0;
    if (check_grid(grid, "grid") != PMF_OK) return 0;
    GridK g = make_grid(*grid);
    return vox_workspace(vox_plan(m, c, g), m);
}

int pmf_voxelize(const pmf_gauss_t *gs, const pmf_grid_t *grid, float trunc_k, float *vol, void *ws,
                 size_t ws_bytes, void *stream) {
    PMF_CHECK(check_gauss(gs));
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_k(trunc_k));
    if (!vol) return fail(PMF_EINVAL, "voxelize: null output");
    GridK g = make_grid(*grid);
    VoxPlan p = vox_plan(gs->m, gs->c, g);
    PMF_CHECK(check_ws(ws, ws_bytes, vox_workspace(p, gs->m)));
    return hip_status(launch_voxelize(*gs, g, trunc_k, vol, p, ws, as_stream(stream)), "voxelize");
}

int pmf_voxelize_bwd(const pmf_gauss_t *gs, const pmf_grid_t *grid, float trunc_k,
                     const float *g_vol, const pmf_gauss_grad_t *grad, void *stream) {
    PMF_CHECK(check_gauss(gs));
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_k(trunc_k));
    if (!grad) return fail(PMF_EINVAL, "voxelize_bwd: null gradient struct");
    if (gs->m > 0 && (!g_vol || !grad->mean || !grad->scale || !grad->quat || !grad->value))
        return fail(PMF_EINVAL, "voxelize_bwd: null array");
    GridK g = make_grid(*grid);
    return hip_status(launch_voxelize_bwd(*gs, g, trunc_k, g_vol, *grad, as_stream(stream)),
                      "voxelize_bwd");
}

// ----------------------------------------------------------------- combine
int pmf_combine_dvf(int L, int B, const float *const *bases, const pmf_grid_t *lvl,
                    const float *coeff, int V, const pmf_grid_t *out, float *dvf, void *stream) {
    PMF_CHECK(check_levels(L, B, bases, lvl, "combine"));
    PMF_CHECK(check_grid(out, "output grid"));
    if (V < 1) return fail(PMF_EINVAL, "combine: V must be >= 1");
    if (!coeff || !dvf) return fail(PMF_EINVAL, "combine: null pointer");
    GridK go = make_grid(*out);
    GridK lg[MAXL];
    LevelsK lv = make_levels(L, B, bases, lvl, go, lg);
    return hip_status(launch_combine(lv, coeff, V, go, dvf, as_stream(stream)), "combine");
}

size_t pmf_combine_dvf_bwd_workspace(int L, int B, const pmf_grid_t *lvl, int V,
                                     const pmf_grid_t *out) {
    if (L < 1 || L > MAXL || B < 1 || B > MAXB || !lvl || !out || V < 1) return 0;
    if (check_grid(out, "output grid") != PMF_OK) return 0;
    for (int l = 0; l < L; ++l)
        if (check_grid(&lvl[l], "level grid") != PMF_OK) return 0;
    GridK go = make_grid(*out);
    GridK lg[MAXL];
    const float *dummy[MAXL] = {nullptr, nullptr, nullptr, nullptr};
    LevelsK lv = make_levels(L, B, dummy, lvl, go, lg);
    return combine_bwd_workspace(lv, lg, V, go);
}

int pmf_combine_dvf_bwd(int L, int B, const float *const *bases, const pmf_grid_t *lvl,
                        const float *coeff, int V, const pmf_grid_t *out, const float *g_dvf,
                        float *const *g_bases, float *g_coeff, void *ws, size_t ws_bytes,
                        void *stream) {
    PMF_CHECK(check_levels(L, B, bases, lvl, "combine_bwd"));
    PMF_CHECK(check_grid(out, "output grid"));
    if (V < 1) return fail(PMF_EINVAL, "combine_bwd: V must be >= 1");
    if (!coeff || !g_dvf || !g_bases || !g_coeff) return fail(PMF_EINVAL, "combine_bwd: null pointer");
    for (int l = 0; l < L; ++l)
        if (!g_bases[l]) return fail(PMF_EINVAL, "combine_bwd: null g_bases[%d]", l);
    GridK go = make_grid(*out);
    GridK lg[MAXL];
    LevelsK lv = make_levels(L, B, bases, lvl, go, lg);
    PMF_CHECK(check_ws(ws, ws_bytes, combine_bwd_workspace(lv, lg, V, go)));
    return hip_status(
        launch_combine_bwd(lv, lg, coeff, V, go, g_dvf, g_bases, g_coeff, ws, as_stream(stream)),
        "combine_bwd");
}

// -------------------------------------------------------------------- warp
int pmf_warp(const float *ref, const pmf_grid_t *grid, const float *dvf, int V, float *out,
             void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    if (V < 1) return fail(PMF_EINVAL, "warp: V must be >= 1");
    if (!ref || !dvf || !out) return fail(PMF_EINVAL, "warp: null pointer");
    GridK g = make_grid(*grid);
    return hip_status(launch_warp(ref, g, dvf, V, out, as_stream(stream)), "warp");
}

size_t pmf_warp_bwd_workspace(const pmf_grid_t *grid) {
    if (!grid || grid->n[0] < 1 || grid->n[1] < 1 || grid->n[2] < 1) return 0;
    return warp_bwd_workspace(make_grid(*grid));
}

int pmf_warp_bwd(const float *ref, const pmf_grid_t *grid, const float *dvf, int V,
                 const float *g_out, float *g_ref, float *g_dvf, void *ws, size_t ws_bytes,
                 void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    if (V < 1) return fail(PMF_EINVAL, "warp_bwd: V must be >= 1");
    if (!ref || !dvf || !g_out || !g_ref || !g_dvf) return fail(PMF_EINVAL, "warp_bwd: null pointer");
    GridK g = make_grid(*grid);
    PMF_CHECK(check_ws(ws, ws_bytes, warp_bwd_workspace(g)));
    return hip_status(launch_warp_bwd(ref, g, dvf, V, g_out, g_ref, g_dvf, ws, as_stream(stream)),
                      "warp_bwd");
}

// -------------------------------------------------------------- projection
int pmf_project(const float *vol, int64_t vol_stride, const pmf_grid_t *grid,
                const pmf_cone_t *cone, const float *angles, int V, float *proj, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_cone(cone, grid));
    if (V < 1) return fail(PMF_EINVAL, "project: V must be >= 1");
    if (!vol || !angles || !proj) return fail(PMF_EINVAL, "project: null pointer");
    if (vol_stride < 0) return fail(PMF_EINVAL, "project: vol_stride < 0");
    GridK g = make_grid(*grid);
    if (vol_stride != 0 && vol_stride < grid_size(g))
        return fail(PMF_EINVAL, "project: vol_stride must be 0 or >= N");
    ConeK c = make_cone(*cone, g);
    return hip_status(launch_project(vol, vol_stride, g, c, angles, V, proj, as_stream(stream)),
                      "project");
}

size_t pmf_project_bwd_workspace(const pmf_grid_t *grid, const pmf_cone_t *cone, int V) {
    if (!grid || !cone || V < 1 || cone->nu < 1 || cone->nv < 1) return 0;
    for (int a = 0; a < 3; ++a)
        if (grid->n[a] < 1) return 0;
    return project_bwd_workspace(make_grid(*grid), *cone, V);
}

int pmf_project_bwd(const float *g_proj, const pmf_grid_t *grid, const pmf_cone_t *cone,
                    const float *angles, int V, float *g_vol, int64_t vol_stride, void *ws,
                    size_t ws_bytes, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_cone(cone, grid));
    if (V < 1) return fail(PMF_EINVAL, "project_bwd: V must be >= 1");
    if (!g_proj || !angles || !g_vol) return fail(PMF_EINVAL, "project_bwd: null pointer");
    GridK g = make_grid(*grid);
    if (vol_stride != 0 && vol_stride < grid_size(g))
        return fail(PMF_EINVAL, "project_bwd: vol_stride must be 0 or >= N");
    PMF_CHECK(check_ws(ws, ws_bytes, project_bwd_workspace(g, *cone, V)));
    ConeK c = make_cone(*cone, g);
    return hip_status(
        launch_project_bwd(g_proj, g, c, angles, V, g_vol, vol_stride, ws, as_stream(stream)),
        "project_bwd");
}

// -------------------------------------------------------------------- loss
size_t pmf_l2_loss_workspace(int64_t npix, int V) {
    if (npix < 1 || V < 1) return 0;
    return l2_workspace(npix, V);
}

int pmf_l2_loss(const float *proj, const float *target, int64_t npix, int V, float *loss,
                float *g_proj, void *ws, size_t ws_bytes, void *stream) {
    if (npix < 1 || V < 1) return fail(PMF_EINVAL, "l2_loss: npix and V must be >= 1");
    if (!proj || !target || !loss) return fail(PMF_EINVAL, "l2_loss: null pointer");
    PMF_CHECK(check_ws(ws, ws_bytes, l2_workspace(npix, V)));
    return hip_status(launch_l2(proj, target, npix, V, loss, g_proj, ws, as_stream(stream)),
                      "l2_loss");
}

// --------------------------------------------------------- FDK initialisation
size_t pmf_fdk_workspace(const pmf_cone_t *cone, int V) {
    if (!cone || V < 1 || cone->nu < 1 || cone->nv < 1) return 0;
    return fdk_workspace(*cone, V);
}

int pmf_fdk(const float *proj, const pmf_cone_t *cone, const float *angles, int V,
            const pmf_grid_t *grid, float *vol, void *ws, size_t ws_bytes, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_cone(cone, grid));
    if (V < 1 || V > 65535) return fail(PMF_EINVAL, "fdk: V must be in [1, 65535]");
    if (cone->nu > 4096) return fail(PMF_EUNSUPPORTED, "fdk: detector rows longer than 4096");
    if (cone->nv > 65535) return fail(PMF_EUNSUPPORTED, "fdk: more than 65535 detector rows");
    if ((int64_t)(cone->nu + 2) * (cone->nv + 2) >= ((int64_t)1 << 27))
        return fail(PMF_EUNSUPPORTED, "fdk: (nu + 2) * (nv + 2) must be < 2^27");
    if (!proj || !angles || !vol) return fail(PMF_EINVAL, "fdk: null pointer");
    PMF_CHECK(check_ws(ws, ws_bytes, fdk_workspace(*cone, V)));
    return hip_status(launch_fdk(proj, *cone, angles, V, make_grid(*grid), vol, ws,
                                 as_stream(stream)),
                      "fdk");
}

int pmf_grid_init(const float *vol, const pmf_grid_t *grid, const int m[3], float scale,
                  float *mean, float *scale_out, float *quat, float *value, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    if (!m) return fail(PMF_EINVAL, "grid_init: null m");
    int64_t M = 1;
    for (int a = 0; a < 3; ++a) {
        if (m[a] < 1 || m[a] > grid->n[a])
            return fail(PMF_EINVAL, "grid_init: m[%d] = %d outside [1, n[%d] = %d]", a, m[a], a,
                        grid->n[a]);
        M *= m[a];
    }
    if (!finite_pos(scale)) return fail(PMF_EINVAL, "grid_init: scale must be > 0");
    if (!vol || !mean || !scale_out || !quat || !value)
        return fail(PMF_EINVAL, "grid_init: null pointer");
    (void)M;
    return hip_status(launch_grid_init(vol, make_grid(*grid), m, scale, mean, scale_out, quat,
                                       value, as_stream(stream)),
                      "grid_init");
}

// ------------------------------------------------------ Stage 1 rasterizer
static int check_rast(const pmf_gauss_t *gs, const pmf_cone_t *c, const float *angles, int V,
                      float k, const char *what) {
    PMF_CHECK(check_gauss(gs));
    if (gs->c != 1) return fail(PMF_EINVAL, "%s: the rasterizer draws one density channel (c = 1)", what);
    PMF_CHECK(check_k(k));
    if (!c) return fail(PMF_EINVAL, "%s: null cone", what);
    if (!(std::isfinite(c->sad) && std::isfinite(c->sdd) && c->sad > 0.0f && c->sdd > c->sad))
        return fail(PMF_EINVAL, "%s: need 0 < SAD < SDD", what);
    if (c->nu < 1 || c->nv < 1) return fail(PMF_EINVAL, "%s: nu, nv must be >= 1", what);
    if (c->nu > 65536 || c->nv > 65536) return fail(PMF_EUNSUPPORTED, "%s: nu, nv <= 65536", what);
    if (!(c->du > 0.0f && c->dv > 0.0f && std::isfinite(c->du) && std::isfinite(c->dv)))
        return fail(PMF_EINVAL, "%s: du, dv must be > 0", what);
    if (!std::isfinite(c->off_u) || !std::isfinite(c->off_v))
        return fail(PMF_EINVAL, "%s: offsets must be finite", what);
    if (V < 1) return fail(PMF_EINVAL, "%s: V must be >= 1", what);
    if (gs->m * V >= ((int64_t)1 << 31) / 16)
        return fail(PMF_EUNSUPPORTED, "%s: m * V too large", what);
    if (!angles) return fail(PMF_EINVAL, "%s: null angles", what);
    return PMF_OK;
}

size_t pmf_rasterize_workspace(int64_t m, const pmf_cone_t *cone, int V) {
    if (m < 0 || !cone || V < 1 || cone->nu < 1 || cone->nv < 1) return 0;
    return rasterize_workspace(m, *cone, V);
}

int pmf_rasterize(const pmf_gauss_t *gs, const pmf_cone_t *cone, const float *angles, int V,
                  float trunc_k, float *proj, void *ws, size_t ws_bytes, void *stream) {
    PMF_CHECK(check_rast(gs, cone, angles, V, trunc_k, "rasterize"));
    if (!proj) return fail(PMF_EINVAL, "rasterize: null proj");
    const int64_t npix = (int64_t)cone->nu * cone->nv * V;
    if (gs->m == 0)
        return hip_status(launch_fill(proj, npix, 0.0f, as_stream(stream)), "rasterize");
    PMF_CHECK(check_ws(ws, ws_bytes, rasterize_workspace(gs->m, *cone, V)));
    return hip_status(launch_rasterize(*gs, *cone, angles, V, trunc_k, proj, ws, as_stream(stream)),
                      "rasterize");
}

static int rasterize_bwd(const pmf_gauss_t *gs, const pmf_cone_t *cone, const float *angles, int V,
                         float trunc_k, const float *g_proj, const pmf_gauss_grad_t *grad,
                         void *ws, size_t ws_bytes, void *stream, bool rebin) {
    PMF_CHECK(check_rast(gs, cone, angles, V, trunc_k, "rasterize_bwd"));
    if (!grad) return fail(PMF_EINVAL, "rasterize_bwd: null gradient struct");
    if (gs->m == 0) return ok();
    if (!g_proj || !grad->mean || !grad->scale || !grad->quat || !grad->value)
        return fail(PMF_EINVAL, "rasterize_bwd: null array");
    PMF_CHECK(check_ws(ws, ws_bytes, rasterize_workspace(gs->m, *cone, V)));
    return hip_status(launch_rasterize_bwd(*gs, *cone, angles, V, trunc_k, g_proj, *grad, ws,
                                           as_stream(stream), rebin),
                      "rasterize_bwd");
}

int pmf_rasterize_bwd(const pmf_gauss_t *gs, const pmf_cone_t *cone, const float *angles, int V,
                      float trunc_k, const float *g_proj, const pmf_gauss_grad_t *grad, void *ws,
                      size_t ws_bytes, void *stream) {
    return rasterize_bwd(gs, cone, angles, V, trunc_k, g_proj, grad, ws, ws_bytes, stream, true);
}

int pmf_rasterize_bwd_binned(const pmf_gauss_t *gs, const pmf_cone_t *cone, const float *angles,
                             int V, float trunc_k, const float *g_proj,
                             const pmf_gauss_grad_t *grad, void *ws, size_t ws_bytes,
                             void *stream) {
    return rasterize_bwd(gs, cone, angles, V, trunc_k, g_proj, grad, ws, ws_bytes, stream, false);
}

// ------------------------------------------------------ Stage 2/3 loss terms
size_t pmf_l1_dssim_loss_workspace(int nu, int nv, int V) {
    if (nu < 1 || nv < 1 || V < 1) return 0;
    return l1_dssim_workspace(nu, nv, V);
}

int pmf_l1_dssim_loss(const float *proj, const float *target, int nu, int nv, int V,
                      float lambda_ssim, float *loss, float *g_proj, void *ws, size_t ws_bytes,
                      void *stream) {
    if (nu < 1 || nv < 1 || V < 1) return fail(PMF_EINVAL, "l1_dssim_loss: nu, nv and V must be >= 1");
    if (!(lambda_ssim >= 0.0f) || !std::isfinite(lambda_ssim))
        return fail(PMF_EINVAL, "l1_dssim_loss: lambda_ssim must be finite and >= 0");
    if (!proj || !target || !loss) return fail(PMF_EINVAL, "l1_dssim_loss: null pointer");
    PMF_CHECK(check_ws(ws, ws_bytes, l1_dssim_workspace(nu, nv, V)));
    return hip_status(launch_l1_dssim(proj, target, nu, nv, V, lambda_ssim, loss, g_proj, ws,
                                      as_stream(stream)),
                      "l1_dssim_loss");
}

size_t pmf_tv_loss_workspace(int D) {
    if (D < 1) return 0;
    return tv_workspace(D);
}

int pmf_tv_loss(const float *vol, const pmf_grid_t *grid, const int32_t *corner, int D,
                float weight, float *loss, float *g_vol, void *ws, size_t ws_bytes, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    if (!corner) return fail(PMF_EINVAL, "tv_loss: null corner");
    if (D < 1) return fail(PMF_EINVAL, "tv_loss: D must be >= 1");
    for (int a = 0; a < 3; ++a)
        if (corner[a] < 0 || (int64_t)corner[a] + D > grid->n[a])
            return fail(PMF_EINVAL, "tv_loss: block [%d, %d) outside axis %d of size %d", corner[a],
                        corner[a] + D, a, grid->n[a]);
    if (!std::isfinite(weight)) return fail(PMF_EINVAL, "tv_loss: weight must be finite");
    if (!vol || !loss) return fail(PMF_EINVAL, "tv_loss: null pointer");
    PMF_CHECK(check_ws(ws, ws_bytes, tv_workspace(D)));
    const int c[3] = {corner[0], corner[1], corner[2]};
    return hip_status(launch_tv(vol, make_grid(*grid), c, D, weight, loss, g_vol, ws,
                                as_stream(stream)),
                      "tv_loss");
}

int pmf_tv_loss_noalloc(const float *vol, const pmf_grid_t *grid, const int32_t *corner, int D,
                        float weight, float *loss, float *g_vol, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    if (!corner) return fail(PMF_EINVAL, "tv_loss_noalloc: null corner");
    if (D < 1) return fail(PMF_EINVAL, "tv_loss_noalloc: D must be >= 1");
    if (D > PMF_TV_NOALLOC_MAX_D)
        return fail(PMF_EUNSUPPORTED,
                    "tv_loss_noalloc: D = %d exceeds the static scratch's maximum %d (use "
                    "pmf_tv_loss with a workspace)",
                    D, PMF_TV_NOALLOC_MAX_D);
    for (int a = 0; a < 3; ++a)
        if (corner[a] < 0 || (int64_t)corner[a] + D > grid->n[a])
            return fail(PMF_EINVAL, "tv_loss_noalloc: block [%d, %d) outside axis %d of size %d",
                        corner[a], corner[a] + D, a, grid->n[a]);
    if (!std::isfinite(weight)) return fail(PMF_EINVAL, "tv_loss_noalloc: weight must be finite");
    if (!vol || !loss) return fail(PMF_EINVAL, "tv_loss_noalloc: null pointer");
    const int c[3] = {corner[0], corner[1], corner[2]};
    return hip_status(launch_tv_noalloc(vol, make_grid(*grid), c, D, weight, loss, g_vol,
                                        as_stream(stream)),
                      "tv_loss_noalloc");
}

size_t pmf_mbc_normality_loss_workspace(int L, int C) {
    if (L < 1 || C < 1) return 0;
    return normality_workspace(L, C);
}

int pmf_mbc_normality_loss(int L, int C, const float *const *bases, const pmf_grid_t *lvl,
                           float weight, float *loss, float *const *g_bases, void *ws,
                           size_t ws_bytes, void *stream) {
    if (L < 1 || C < 1) return fail(PMF_EINVAL, "mbc_normality_loss: L and C must be >= 1");
    if (L > MAXL) return fail(PMF_EUNSUPPORTED, "mbc_normality_loss: L <= 4");
    if (C > 65535) return fail(PMF_EINVAL, "mbc_normality_loss: C too large");
    if (!bases || !lvl || !loss) return fail(PMF_EINVAL, "mbc_normality_loss: null pointer");
    if (!std::isfinite(weight)) return fail(PMF_EINVAL, "mbc_normality_loss: weight must be finite");
    GridK lg[MAXL];
    for (int l = 0; l < L; ++l) {
        if (!bases[l]) return fail(PMF_EINVAL, "mbc_normality_loss: null basis pointer %d", l);
        if (g_bases && !g_bases[l]) return fail(PMF_EINVAL, "mbc_normality_loss: null g_bases[%d]", l);
        PMF_CHECK(check_grid(&lvl[l], "level grid"));
        lg[l] = make_grid(lvl[l]);
    }
    PMF_CHECK(check_ws(ws, ws_bytes, normality_workspace(L, C)));
    return hip_status(launch_normality(L, C, bases, lg, weight, loss, g_bases, ws,
                                       as_stream(stream)),
                      "mbc_normality_loss");
}

// ----------------------------------------------------------------- utility
int pmf_accumulate(float *dst, const float *src, int64_t n, void *stream) {
    if (n < 0) return fail(PMF_EINVAL, "accumulate: n < 0");
    if (n > 0 && (!dst || !src)) return fail(PMF_EINVAL, "accumulate: null pointer");
    return hip_status(launch_accumulate(dst, src, n, as_stream(stream)), "accumulate");
}

int pmf_fill(float *dst, int64_t n, float value, void *stream) {
    if (n < 0) return fail(PMF_EINVAL, "fill: n < 0");
    if (n > 0 && !dst) return fail(PMF_EINVAL, "fill: null pointer");
    return hip_status(launch_fill(dst, n, value, as_stream(stream)), "fill");
}

// --------------------------------------------------------------- profiling
int pmf_profile(int enable) { return profile_enable(enable); }

int pmf_profile_read(const char *kernel, double *total_ms, int64_t *count) {
    if (!kernel || !total_ms || !count) return fail(PMF_EINVAL, "profile_read: null pointer");
    if (profile_read(kernel, total_ms, count) != 0) return fail(PMF_EHIP, "profile_read: event error");
    return ok();
}

size_t pmf_profile_names(char *buf, size_t len) { return profile_names(buf, len); }

// ------------------------------------------------------------ launch shapes
int pmf_tune_candidates(int knob) { return tune_candidates(knob); }

int pmf_tune_get(int knob) {
    if (tune_candidates(knob) == 0) return fail(PMF_EINVAL, "tune_get: unknown knob");
    return tune_get(knob);
}

int pmf_tune_set(int knob, int choice) {
    const int prev = tune_set(knob, choice);
    if (prev < 0) return fail(PMF_EINVAL, "tune_set: unknown knob or choice out of range");
    return prev;
}

int pmf_autotune_project(const float *vol, const pmf_grid_t *grid, const pmf_cone_t *cone,
                         const float *angles, int V, float *proj, const float *g_proj,
                         float *g_vol, void *ws, size_t ws_bytes, int reps, float *ms,
                         void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_cone(cone, grid));
    if (V < 1) return fail(PMF_EINVAL, "autotune: V must be >= 1");
    if (reps < 1) return fail(PMF_EINVAL, "autotune: reps must be >= 1");
    if (!vol || !angles || !proj || !g_proj || !g_vol)
        return fail(PMF_EINVAL, "autotune: null pointer");
    const GridK g = make_grid(*grid);
    PMF_CHECK(check_ws(ws, ws_bytes, project_bwd_workspace(g, *cone, V)));
    const ConeK c = make_cone(*cone, g);
    const int64_t N = grid_size(g);
    hipStream_t st = as_stream(stream);
    const int knobs[2] = {KNOB_PROJECT_TILE, KNOB_BACKPROJECT_BRICK};
    const int prev[2] = {tune_get(knobs[0]), tune_get(knobs[1])};
    const int was_prof = profile_enable(0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int slot = 0;
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
        int best = prev[q];
        float best_ms = INFINITY;
        for (int k = 0; k < tune_candidates(knobs[q]) && e == hipSuccess; ++k) {
            tune_set(knobs[q], k);
            auto run = [&]() {
                return q == 0 ? launch_project(vol, N, g, c, angles, V, proj, st)
                              : launch_project_bwd(g_proj, g, c, angles, V, g_vol, N, ws, st);
            };
            if ((e = run()) != hipSuccess) break;
            if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
            if (e != hipSuccess) break;
            if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float t = 0.0f;
            if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
            t /= (float)reps;
            if (ms) ms[slot] = t;
            ++slot;
            if (t < best_ms) {
                best_ms = t;
                best = k;
            }
        }
        tune_set(knobs[q], best);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    profile_enable(was_prof);
    if (e != hipSuccess) {
        tune_set(knobs[0], prev[0]);
        tune_set(knobs[1], prev[1]);
        return hip_status(e, "autotune_project");
    }
    return ok();
}

// ------------------------------------------- autotuner with a shape cache

int pmf_autotune(const char *cache_path, const float *vol, const pmf_grid_t *grid,
                 const pmf_cone_t *cone, const float *angles, int V, float *proj,
                 const float *g_proj, float *g_vol, void *ws, size_t ws_bytes, int reps, float *ms,
                 int *cached, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_cone(cone, grid));
    if (V < 1) return fail(PMF_EINVAL, "autotune: V must be >= 1");
    if (reps < 1) return fail(PMF_EINVAL, "autotune: reps must be >= 1");
    if (!vol || !angles || !proj || !g_proj || !g_vol)
        return fail(PMF_EINVAL, "autotune: null pointer");
    PMF_CHECK(check_ws(ws, ws_bytes, project_bwd_workspace(make_grid(*grid), *cone, V)));
    if (cached) *cached = 0;
    std::string key;
    if (cache_path) {
        key = autotune_key(grid, cone, V);
        int tile = -1, brick = -1;
        if (autotune_lookup(cache_path, key, tile, brick)) {
            tune_set(KNOB_PROJECT_TILE, tile);
            tune_set(KNOB_BACKPROJECT_BRICK, brick);
            if (cached) *cached = 1;
            return ok();
        }
    }
    const int rc = pmf_autotune_project(vol, grid, cone, angles, V, proj, g_proj, g_vol, ws,
                                        ws_bytes, reps, ms, stream);
    if (rc != PMF_OK || !cache_path) return rc;
    FILE *f = fopen(cache_path, "a");
    if (!f) return fail(PMF_EINVAL, "autotune: cannot append to the cache %s", cache_path);
    const int w = fprintf(f, "%s\t%d\t%d\n", key.c_str(), tune_get(KNOB_PROJECT_TILE),
                          tune_get(KNOB_BACKPROJECT_BRICK));
    if (fclose(f) != 0 || w < 0)
        return fail(PMF_EINVAL, "autotune: cannot write the cache %s", cache_path);
    return ok();
}

// ------------------------------------------------------------ graph capture
struct pmf_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int64_t nodes, kernels;
};

int pmf_graph_capture(void *stream, pmf_record_fn record, void *user, pmf_graph_t **graph) {
    if (!graph) return fail(PMF_EINVAL, "graph_capture: null output");
    *graph = nullptr;
    if (!stream)
        return fail(PMF_EINVAL, "graph_capture: the legacy default stream cannot be captured");
    if (!record) return fail(PMF_EINVAL, "graph_capture: null record function");
    hipStream_t s = as_stream(stream);
    // profiling events would become graph nodes: off while recording
    const int was_prof = profile_enable(0);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        profile_enable(was_prof);
        return hip_status(e, "graph_capture: begin");
    }
    const int rc = record(user, stream);
    const std::string rec_err = rc != PMF_OK ? g_err : std::string();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    profile_enable(was_prof);
    if (rc != PMF_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc != PMF_OK) return fail(rc, "graph_capture: recording failed: %s", rec_err.c_str());
        return hip_status(e, "graph_capture: end");
    }
    size_t n = 0;
    e = hipGraphGetNodes(g, nullptr, &n);
    std::vector<hipGraphNode_t> nodes(n);
    if (e == hipSuccess && n) e = hipGraphGetNodes(g, nodes.data(), &n);
    int64_t kernels = 0;
    for (size_t i = 0; i < n && e == hipSuccess; ++i) {
        hipGraphNodeType t;
        e = hipGraphNodeGetType(nodes[i], &t);
        if (e != hipSuccess) break;
        if (t == hipGraphNodeTypeMemset) {
            (void)hipGraphDestroy(g);
            return fail(PMF_EUNSUPPORTED, "graph_capture: the recorded work holds a memset node");
        }
        if (t == hipGraphNodeTypeKernel) ++kernels;
    }
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_status(e, "graph_capture: instantiate");
    }
    *graph = new pmf_graph{g, x, (int64_t)n, kernels};
    return ok();
}

int pmf_graph_replay(const pmf_graph_t *graph, void *stream) {
    if (!graph) return fail(PMF_EINVAL, "graph_replay: null graph");
    return hip_status(hipGraphLaunch(graph->exec, as_stream(stream)), "graph_replay");
}

int64_t pmf_graph_kernel_count(const pmf_graph_t *graph) {
    return graph ? graph->kernels : -1;
}

int pmf_graph_destroy(pmf_graph_t *graph) {
    if (!graph) return ok();
    hipError_t e = hipGraphExecDestroy(graph->exec);
    const hipError_t e2 = hipGraphDestroy(graph->graph);
    if (e == hipSuccess) e = e2;
    delete graph;
    return hip_status(e, "graph_destroy");
}

// ------------------------------------------------------ fused motion path
size_t pmf_warp_project_workspace(int L, int B, const pmf_grid_t *lvl, int V,
                                  const pmf_grid_t *grid, const pmf_cone_t *cone) {
    (void)lvl;
    if (L < 1 || L > MAXL || B < 1 || B > MAXB || V < 1 || !grid || !cone) return 0;
    if (check_grid(grid, "grid") != PMF_OK) return 0;
    GridK g = make_grid(*grid);
    LevelsK lv{};
    lv.L = L;
    lv.B = B;
    return warp_project_workspace(lv, V, g, *cone);
}

int pmf_warp_project(const float *ref, const pmf_grid_t *grid, int L, int B,
                     const float *const *bases, const pmf_grid_t *lvl, const float *coeff, int V,
                     const pmf_cone_t *cone, const float *angles, float *proj, void *ws,
                     size_t ws_bytes, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_levels(L, B, bases, lvl, "warp_project"));
    PMF_CHECK(check_cone(cone, grid));
    if (V < 1) return fail(PMF_EINVAL, "warp_project: V must be >= 1");
    if (!ref || !coeff || !angles || !proj) return fail(PMF_EINVAL, "warp_project: null pointer");
    GridK g = make_grid(*grid);
    GridK lg[MAXL];
    LevelsK lv = make_levels(L, B, bases, lvl, g, lg);
    PMF_CHECK(check_ws(ws, ws_bytes, warp_project_workspace(lv, V, g, *cone)));
    ConeK c = make_cone(*cone, g);
    return hip_status(
        launch_warp_project(ref, g, lv, coeff, V, c, angles, proj, ws, as_stream(stream)),
        "warp_project");
}

size_t pmf_warp_project_bwd_workspace(int L, int B, const pmf_grid_t *lvl, int V,
                                      const pmf_grid_t *grid, const pmf_cone_t *cone) {
    if (L < 1 || L > MAXL || B < 1 || B > MAXB || V < 1 || !grid || !cone || !lvl) return 0;
    if (check_grid(grid, "grid") != PMF_OK) return 0;
    for (int l = 0; l < L; ++l)
        if (check_grid(&lvl[l], "level grid") != PMF_OK) return 0;
    GridK g = make_grid(*grid);
    GridK lg[MAXL];
    const float *dummy[MAXL] = {nullptr, nullptr, nullptr, nullptr};
    LevelsK lv = make_levels(L, B, dummy, lvl, g, lg);
    return warp_project_bwd_workspace(lv, lg, V, g, *cone);
}

int pmf_warp_project_bwd(const float *ref, const pmf_grid_t *grid, int L, int B,
                         const float *const *bases, const pmf_grid_t *lvl, const float *coeff,
                         int V, const pmf_cone_t *cone, const float *angles, const float *g_proj,
                         float *g_ref, float *const *g_bases, float *g_coeff, void *ws,
                         size_t ws_bytes, void *stream) {
    PMF_CHECK(check_grid(grid, "grid"));
    PMF_CHECK(check_levels(L, B, bases, lvl, "warp_project_bwd"));
    PMF_CHECK(check_cone(cone, grid));
    if (V < 1) return fail(PMF_EINVAL, "warp_project_bwd: V must be >= 1");
    if (!ref || !coeff || !angles || !g_proj || !g_ref || !g_bases || !g_coeff)
        return fail(PMF_EINVAL, "warp_project_bwd: null pointer");
    for (int l = 0; l < L; ++l)
        if (!g_bases[l]) return fail(PMF_EINVAL, "warp_project_bwd: null g_bases[%d]", l);
    GridK g = make_grid(*grid);
    GridK lg[MAXL];
    LevelsK lv = make_levels(L, B, bases, lvl, g, lg);
    PMF_CHECK(check_ws(ws, ws_bytes, warp_project_bwd_workspace(lv, lg, V, g, *cone)));
    ConeK c = make_cone(*cone, g);
    return hip_status(launch_warp_project_bwd(ref, g, lv, lg, coeff, V, c, angles, g_proj, g_ref,
                                              g_bases, g_coeff, ws, as_stream(stream)),
                      "warp_project_bwd");
}

// ------------------------------------------------ ragged batch of scans
}  // extern "C"

namespace {

static_assert(PMF_MAX_SCANS == MAXS && PMF_MAX_LEVELS == MAXL, "table sizes");

// Validates scan k's forward fields; fills its kernel descriptors.
int scan_fwd(int L, int B, const pmf_scan_t &sc, int k, GridK &g, GridK *lg, LevelsK &lv,
             ConeK &c) {
    char what[64];
    snprintf(what, sizeof what, "scan %d", k);
    PMF_CHECK(check_grid(&sc.grid, what));
    PMF_CHECK(check_levels(L, B, sc.bases, sc.lvl, what));
    PMF_CHECK(check_cone(&sc.cone, &sc.grid));
    if (sc.V < 1) return fail(PMF_EINVAL, "%s: V must be >= 1", what);
    if (!sc.ref || !sc.coeff || !sc.angles) return fail(PMF_EINVAL, "%s: null pointer", what);
    g = make_grid(sc.grid);
    lv = make_levels(L, B, sc.bases, sc.lvl, g, lg);
    c = make_cone(sc.cone, g);
    return PMF_OK;
}

int check_scans(const pmf_scan_t *scans, int n) {
    if (!scans) return fail(PMF_EINVAL, "scans: null");
    if (n < 1 || n > MAXS) return fail(PMF_EINVAL, "scans: n_scans must be in [1, %d]", MAXS);
    return PMF_OK;
}

}  // namespace

extern "C" {

size_t pmf_warp_project_scans_workspace(int L, int B, const pmf_scan_t *scans, int n) {
    if (!scans || n < 1 || n > MAXS) return 0;
    size_t total = 0;
    for (int k = 0; k < n; ++k) {
        size_t w = pmf_warp_project_workspace(L, B, scans[k].lvl, scans[k].V, &scans[k].grid,
                                              &scans[k].cone);
        if (w == 0) return 0;
        total += align256(w);
    }
    return total;
}

int pmf_warp_project_scans(int L, int B, const pmf_scan_t *scans, int n, void *ws,
                           size_t ws_bytes, void *stream) {
    PMF_CHECK(check_scans(scans, n));
    WPJob jobs[MAXS];
    char *w = (char *)ws;
    size_t need = 0;
    for (int k = 0; k < n; ++k) {
        const pmf_scan_t &sc = scans[k];
        GridK lg[MAXL];
        WPJob &j = jobs[k];
        PMF_CHECK(scan_fwd(L, B, sc, k, j.g, lg, j.lv, j.c));
        if (!sc.proj) return fail(PMF_EINVAL, "scan %d: null proj", k);
        j.ref = sc.ref;
        j.coeff = sc.coeff;
        j.V = sc.V;
        j.angles = sc.angles;
        j.proj = sc.proj;
        j.ws = w ? w + need : nullptr;
        need += align256(warp_project_workspace(j.lv, sc.V, j.g, sc.cone));
    }
    PMF_CHECK(check_ws(ws, ws_bytes, need));
    return hip_status(launch_warp_project_jobs(jobs, n, as_stream(stream)), "warp_project_scans");
}

size_t pmf_warp_project_bwd_scans_workspace(int L, int B, const pmf_scan_t *scans, int n) {
    if (!scans || n < 1 || n > MAXS) return 0;
    size_t total = 0;
    for (int k = 0; k < n; ++k) {
        size_t w = pmf_warp_project_bwd_workspace(L, B, scans[k].lvl, scans[k].V, &scans[k].grid,
                                                  &scans[k].cone);
        if (w == 0) return 0;
        total += align256(w);
    }
    return total;
}

int pmf_warp_project_bwd_scans(int L, int B, const pmf_scan_t *scans, int n, void *ws,
                               size_t ws_bytes, void *stream) {
    PMF_CHECK(check_scans(scans, n));
    WPBJob jobs[MAXS];
    char *w = (char *)ws;
    size_t need = 0;
    for (int k = 0; k < n; ++k) {
        const pmf_scan_t &sc = scans[k];
        WPBJob &j = jobs[k];
        PMF_CHECK(scan_fwd(L, B, sc, k, j.g, j.lvl_grids, j.lv, j.c));
        if (!sc.g_proj || !sc.g_ref || !sc.g_coeff)
            return fail(PMF_EINVAL, "scan %d: null adjoint pointer", k);
        for (int l = 0; l < MAXL; ++l) {
            if (l < L && !sc.g_bases[l]) return fail(PMF_EINVAL, "scan %d: null g_bases[%d]", k, l);
            j.g_bases[l] = l < L ? sc.g_bases[l] : nullptr;
        }
        j.ref = sc.ref;
        j.coeff = sc.coeff;
        j.V = sc.V;
        j.angles = sc.angles;
        j.g_proj = sc.g_proj;
        j.g_ref = sc.g_ref;
        j.g_coeff = sc.g_coeff;
        j.ws = w ? w + need : nullptr;
        need += align256(warp_project_bwd_workspace(j.lv, j.lvl_grids, sc.V, j.g, sc.cone));
    }
    PMF_CHECK(check_ws(ws, ws_bytes, need));
    return hip_status(launch_warp_project_bwd_jobs(jobs, n, as_stream(stream)),
                      "warp_project_bwd_scans");
}

}  // extern "C"
