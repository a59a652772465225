// vr_api.hip -- the C ABI (include/vr.h): argument and state checks, camera
// basis, volume layout description, launch shapes, and the host side of the
// brick, batch and tuning paths.  Every device buffer is the caller's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vr_ctx.h"

using namespace vr;

static thread_local std::string g_err;

int vr_fail(const vr_ctx *ctx, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) const_cast<vr_ctx *>(ctx)->err = buf;
    g_err = buf;
    return code;
}
#define fail vr_fail

int64_t vr_align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

static int ok(vr_ctx *ctx) {
    if (ctx) ctx->err.clear();
    return VR_OK;
}

static int no_device(vr_ctx *ctx) {
    return fail(ctx, VR_EDEVICE, "context was created without a device");
}

int vr_dev_check(vr_ctx *ctx, hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(ctx, VR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return ok(ctx);
}
#define dev_check vr_dev_check

void *vr_stage(vr_ctx *ctx, size_t bytes) {
    if (ctx->stage_pending) {
        if (hipEventSynchronize(ctx->stage_done) != hipSuccess) return nullptr;
        ctx->stage_pending = false;
    }
    if (bytes > ctx->stage_bytes) {
        if (ctx->stage) (void)hipHostFree(ctx->stage);
        ctx->stage = nullptr;
        ctx->stage_bytes = 0;
        size_t cap = std::max<size_t>(bytes, 64 * 1024);
        if (hipHostMalloc(&ctx->stage, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
        ctx->stage_bytes = cap;
    }
    return ctx->stage;
}

hipError_t vr_stage_copy(vr_ctx *ctx, void *dst, size_t bytes, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(dst, ctx->stage, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    if (!ctx->stage_done) {
        e = hipEventCreateWithFlags(&ctx->stage_done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    e = hipEventRecord(ctx->stage_done, s);
    if (e == hipSuccess) ctx->stage_pending = true;
    return e;
}

static int64_t esize(int32_t dt) { return dt == VR_F32 ? 4 : 2; }

// ---------------------------------------------------------------------------
// camera basis (host, FP64)
// ---------------------------------------------------------------------------
namespace vr {
bool make_cam(const vr_camera &c, CamDev *o) {
    double f[3], r[3], u[3];
    for (int a = 0; a < 3; ++a) f[a] = c.target[a] - c.eye[a];
    double nf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(nf > 0) || !std::isfinite(nf)) return false;
    for (int a = 0; a < 3; ++a) f[a] /= nf;
    r[0] = f[1] * c.up[2] - f[2] * c.up[1];
    r[1] = f[2] * c.up[0] - f[0] * c.up[2];
    r[2] = f[0] * c.up[1] - f[1] * c.up[0];
    double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(nr > 0) || !std::isfinite(nr)) return false;
    for (int a = 0; a < 3; ++a) r[a] /= nr;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    for (int a = 0; a < 3; ++a) {
        o->eye[a] = c.eye[a];
        o->f[a] = f[a];
        o->r[a] = r[a];
        o->u[a] = u[a];
    }
    o->W = c.full_w;
    o->H = c.full_h;
    if (c.kind == VR_PERSPECTIVE) {
        double th = std::tan(c.fovy_deg * M_PI / 360.0);
        o->a = th * (double)c.full_w / (double)c.full_h;
        o->b = th;
    } else {
        o->a = c.half_w;
        o->b = c.half_h;
    }
    o->kind = c.kind;
    o->tile_x0 = c.tile_x0;
    o->tile_y0 = c.tile_y0;
    o->tile_w = c.tile_w;
    o->tile_h = c.tile_h;
    o->pad = 0;
    return true;
}
}  // namespace vr

static int check_camera(vr_ctx *ctx, const vr_camera *c, CamDev *out) {
    if (!c) return fail(ctx, VR_EINVAL, "camera is NULL");
    if (c->kind != VR_ORTHO && c->kind != VR_PERSPECTIVE) return fail(ctx, VR_EINVAL, "camera kind %d", c->kind);
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->eye[a]) || !std::isfinite(c->target[a]) || !std::isfinite(c->up[a]))
            return fail(ctx, VR_EINVAL, "camera has a non-finite coordinate");
    if (c->full_w <= 0 || c->full_h <= 0) return fail(ctx, VR_EINVAL, "full frame %dx%d", c->full_w, c->full_h);
    if (c->tile_w <= 0 || c->tile_h <= 0 || c->tile_x0 < 0 || c->tile_y0 < 0 ||
        (int64_t)c->tile_x0 + c->tile_w > c->full_w || (int64_t)c->tile_y0 + c->tile_h > c->full_h)
        return fail(ctx, VR_EINVAL, "viewport (%d,%d,%d,%d) outside the %dx%d frame", c->tile_x0, c->tile_y0,
                    c->tile_w, c->tile_h, c->full_w, c->full_h);
    if ((int64_t)c->tile_w * c->tile_h > (int64_t)1 << 31) return fail(ctx, VR_EINVAL, "viewport too large");
    if (c->kind == VR_PERSPECTIVE && !(c->fovy_deg > 0 && c->fovy_deg < 180))
        return fail(ctx, VR_EINVAL, "fovy %g not in (0, 180)", c->fovy_deg);
    if (c->kind == VR_ORTHO && !(c->half_w > 0 && c->half_h > 0 && std::isfinite(c->half_w) && std::isfinite(c->half_h)))
        return fail(ctx, VR_EINVAL, "orthographic half extents must be > 0");
    CamDev cd{};
    if (!make_cam(*c, &cd)) return fail(ctx, VR_EINVAL, "degenerate camera basis (eye == target or up parallel to the view)");
    if (out) *out = cd;
    return VR_OK;
}

int vr_check_params(vr_ctx *ctx, const vr_render_params *p) {
#define check_params vr_check_params
    if (!p) return fail(ctx, VR_EINVAL, "params is NULL");
    if (p->mode != VR_COMPOSITE && p->mode != VR_MIP) return fail(ctx, VR_EINVAL, "mode %d", p->mode);
    if (p->filter != VR_TRILINEAR && p->filter != VR_NEAREST) return fail(ctx, VR_EINVAL, "filter %d", p->filter);
    // fixed-point positions resolve 2^-32 voxel: keep the per-sample increment
    // far above that, and the sample count of any ray within int32
    if (!(p->step >= 1e-4) || !std::isfinite(p->step) || p->step > 1e6)
        return fail(ctx, VR_EINVAL, "step %g must be in [1e-4, 1e6]", p->step);
    if (!(p->ert_alpha > 0)) return fail(ctx, VR_EINVAL, "ert_alpha %g must be > 0", (double)p->ert_alpha);
    if (p->transmittance < 0 || p->transmittance > 2) return fail(ctx, VR_EINVAL, "transmittance %d", p->transmittance);
    return VR_OK;
}

int vr_need_state(vr_ctx *ctx, bool lut_needed, bool streamed_ok) {
#define need_state vr_need_state
    if (!ctx) return fail(nullptr, VR_EINVAL, "context is NULL");
    if (ctx->device < 0 && ctx->vol_loaded) return no_device(ctx);
    if (!ctx->vol_loaded) return fail(ctx, VR_ESTATE, "no volume loaded");
    if (ctx->st.on && !streamed_ok)
        return fail(ctx, VR_EUNSUPPORTED, "the volume is streamed from host memory: render it with vr_render_bricks");
    if (!ctx->has_camera) return fail(ctx, VR_ESTATE, "no camera set");
    if (lut_needed && !ctx->has_lut) return fail(ctx, VR_ESTATE, "no transfer function set");
    return VR_OK;
}

// Maximum samples of any ray through the cube.
static int64_t max_samples(const VolDev &v, double step) {
    double diag = std::sqrt((double)v.nx * v.nx + (double)v.ny * v.ny + (double)v.nz * v.nz);
    return (int64_t)std::ceil(diag / step) + 2;
}

static void select_copy(VolDev &v, const CamDev &c, int32_t forced);

MarchArgs vr_march_args(vr_ctx *ctx, const vr_render_params *p, const CamDev &cam) {
#define march_args vr_march_args
    MarchArgs a{};
    a.cam = cam;
    a.vol = ctx->vol;
    a.lut = ctx->lut;
    a.step = p->step;
    a.ert = p->ert_alpha < 1.0f ? 1 : 0;
    a.thr = 1.0f - p->ert_alpha;
    if (p->transmittance == VR_TRANS_PRODUCT) a.trans = 0;
    else if (p->transmittance == VR_TRANS_LOG) a.trans = 1;
    else a.trans = a.ert ? 2 : 1;
    a.packet_w = ctx->tune.packet_w;
    a.packet_h = ctx->tune.packet_h;
    a.waves = ctx->tune.waves_per_group;
    a.groups_x = (cam.tile_w + a.packet_w - 1) / a.packet_w;
    a.unroll = ctx->tune.unroll;
    a.order = ctx->tune.order;
    select_copy(a.vol, cam, ctx->tune.copy);
    return a;
}

// Depth in voxels below which no ray of a composite can stop early: with
// every sample's opacity at most amax, A after n samples is at most
// 1 - (1 - amax)^n, so A >= tau needs n >= log(1 - tau) / log(1 - amax).
static double min_stop_depth(const vr_ctx *ctx, const vr_render_params *p) {
    if (p->ert_alpha >= 1.0f || ctx->lut_amax <= 0.0f) return INFINITY;
    if (ctx->lut_amax >= 1.0f || p->ert_alpha <= 0.0f) return 0.0;
    const double n = std::log(1.0 - (double)p->ert_alpha) / std::log1p(-(double)ctx->lut_amax);
    return std::ceil(n) * p->step;
}

// The LDS-staged kernel serves one-brick layouts; the direct-gather kernel
// walks multi-brick layouts and serves as the fallback.  Automatic choice:
// long rays stage voxel boxes in LDS: MIP, composites without early
// termination, and composites whose table is transparent enough that no ray
// can stop within its first 64 voxels (min_stop_depth); other
// early-terminating composites, whose rays may stop after a few samples,
// gather directly.  Both kernels give bit-identical images, so the choice
// only moves time.
static bool use_slab_path(const vr_ctx *ctx, const vr_render_params *p) {
    if (!ctx->vol.single) return false;
    if (ctx->tune.path == 1 || ctx->tune.path == 3 || ctx->tune.waves_per_group < 4) return false;
    if (ctx->tune.path == 2) return true;
    return p->mode == VR_MIP || p->ert_alpha >= 1.0f || min_stop_depth(ctx, p) >= 64.0;
}

// The compacting direct kernel (path 3) on one-brick layouts.
static bool use_compact_path(const vr_ctx *ctx) {
    return ctx->vol.single && ctx->tune.path == 3 && ctx->tune.waves_per_group <= 4;
}

// MIP in object order (path 4) on one-brick layouts; it keeps per-pixel ray
// records in the workspace.  The automatic choice (path 0 with the automatic
// LDS budget) takes it for views whose far slab boxes, even in the best
// orientation copy, exceed 50 KiB (views oblique to the axes): there the
// blocks read each voxel about once, while the bundles' boxes overlap most.
// The object-order frame costs about the same at every angle; the bundles'
// frame grows with their box sizes, and 50 KiB is where the two cross on the
// orbit views of an 8 GiB cube at 1920x1080.
static bool use_block_path(const vr_ctx *ctx, const vr_render_params *p) {
    if (!ctx->vol.single || p->mode != VR_MIP || !ctx->has_camera) return false;
    if (ctx->tune.path == 4) return true;
    if (ctx->tune.path != 0 || ctx->tune.lds_kib != 0 || ctx->tune.waves_per_group < 4) return false;
    double best = 1e300;
    for (int o = 0; o < (ctx->vol.orients == 3 ? 3 : 1); ++o) {
        VolDev v = ctx->vol;
        apply_copy(v, o);
        best = std::min(best, vr_box_estimate_kib(ctx->camd, v, ctx->tune.packet_w,
                                                  ctx->tune.packet_h * ctx->tune.waves_per_group));
    }
    return best > 50.0;
}

// Automatic LDS budget of the slab path (tuning lds_kib = 0).  Two
// workgroups per CU (64 KiB each) keep more waves in flight; a view whose
// bundles need very wide boxes (oblique to all three axes) would march its
// far slabs with direct gathers at that budget, so it gets one workgroup per
// CU with 144 KiB.  The estimate: the box at slab thickness 2 near the far
// face of the cube, for bundles spread over the viewport.
double vr_box_estimate_kib(const CamDev &c, const VolDev &v, int32_t bw, int32_t bh) {
    const double N[3] = {(double)v.nx, (double)v.ny, (double)v.nz};
    const int32_t L = 2;
    double worst = 0.0;
    const int32_t sx = std::max(bw, c.tile_w / 12), sy = std::max(bh, c.tile_h / 9);
    for (int32_t y0 = 0; y0 < c.tile_h; y0 += sy) {
        for (int32_t x0 = 0; x0 < c.tile_w; x0 += sx) {
            const int32_t x1 = std::min(x0 + bw, c.tile_w) - 1, y1 = std::min(y0 + bh, c.tile_h) - 1;
            double o[4][3], d[4][3], dc[3] = {0, 0, 0};
            for (int k = 0; k < 4; ++k) {
                cam_ray(c, c.tile_x0 + ((k & 1) ? x1 : x0), c.tile_y0 + ((k & 2) ? y1 : y0), o[k][0], o[k][1],
                        o[k][2], d[k][0], d[k][1], d[k][2]);
                for (int a = 0; a < 3; ++a) dc[a] += d[k][a];
            }
            int w = 0;
            for (int a = 1; a < 3; ++a)
                if (std::fabs(dc[a]) > std::fabs(dc[w])) w = a;
            // the bundle's central line against the cube
            double tn = -1e300, tf = 1e300;
            bool hit = true;
            for (int a = 0; a < 3; ++a) {
                const double oa = (o[0][a] + o[3][a]) * 0.5, da = dc[a] * 0.25;
                if (da == 0.0) { hit = hit && oa >= 0.0 && oa <= N[a]; continue; }
                const double ta = (0.0 - oa) / da, tb = (N[a] - oa) / da;
                tn = std::max(tn, std::min(ta, tb));
                tf = std::min(tf, std::max(ta, tb));
            }
            if (!hit || !(tf > tn) || std::fabs(dc[w]) < 0.8) continue;
            const double t = tf - 0.02 * (tf - tn);
            const double pw = (o[0][w] + o[3][w]) * 0.5 + t * dc[w] * 0.25;
            const double lo = dc[w] > 0 ? pw - L : pw;
            double ext[3];
            ext[w] = L + 1;
            for (int a = 0; a < 3; ++a) {
                if (a == w) continue;
                double mn = 1e300, mx = -1e300;
                for (int k = 0; k < 4; ++k) {
                    for (int e = 0; e < 2; ++e) {
                        const double p = lo + 0.5 + e * L;
                        const double q = o[k][a] + (p - o[k][w]) / d[k][w] * d[k][a];
                        mn = std::min(mn, q);
                        mx = std::max(mx, q);
                    }
                }
                ext[a] = std::floor(mx) - std::floor(mn) + 2.0;
            }
            const double epc = v.dtype == VR_F32 ? 4.0 : 8.0;           // elements per 16-byte chunk
            ext[v.ori] = std::ceil((ext[v.ori] + epc) / epc) * epc;       // whole chunks, misaligned start
            worst = std::max(worst, ext[0] * ext[1] * ext[2] * 4.0 / 1024.0);
        }
    }
    return worst;
}

int32_t vr_auto_box_kib(const CamDev &c, const VolDev &v, int32_t bw, int32_t bh) {
    return vr_box_estimate_kib(c, v, bw, bh) > 100.0 ? 144 : 64;
}

// Workspace bytes of the costliest-first bundle order (tuning order 3 on
// the LDS-staged path, without save_for_backward), else 0.
static int64_t order_bytes(const vr_ctx *ctx, const vr_render_params *p) {
    if (ctx->tune.order != 3 || p->save_for_backward || use_compact_path(ctx) || !use_slab_path(ctx, p)) return 0;
    return slab_order_bytes(ctx->cam.tile_w, ctx->cam.tile_h, ctx->tune.packet_w,
                            ctx->tune.packet_h * ctx->tune.waves_per_group);
}

// ws: the caller's workspace when it holds the bundle order (order_bytes),
// else NULL (the bundles then run in hardware order).
static hipError_t dispatch_render(vr_ctx *ctx, const MarchArgs &a, const vr_render_params *p, hipStream_t s,
                                  void *ws = nullptr) {
    if (use_compact_path(ctx)) return launch_march_compact(a, p->mode, p->filter, ctx->tune.persistent_groups, s);
    if (use_slab_path(ctx, p)) {
        const int32_t bh = a.packet_h * a.waves;
        const int32_t kib = ctx->tune.lds_kib > 0 ? ctx->tune.lds_kib
                                                  : vr_auto_box_kib(a.cam, a.vol, a.packet_w, bh);
        int32_t cap = kib * 1024 / 4;
        MarchArgs b = a;
        b.tile_perm = nullptr;
        b.tile_key = nullptr;
        if (ws && a.order == 3) {
            const int64_t n = (int64_t)((a.cam.tile_w + a.packet_w - 1) / a.packet_w) * ((a.cam.tile_h + bh - 1) / bh);
            b.tile_perm = (int32_t *)ws;
            b.tile_key = (uint8_t *)ws + (n * 4 + 255) / 256 * 256;
        }
        return launch_slab(b, p->mode, p->filter, a.packet_w, bh, cap, ctx->tune.slab_max, s);
    }
    if (ctx->tune.path == 0 && ctx->vol.single && p->mode == VR_COMPOSITE) {
        // the automatic shape of the direct kernel for early-stopping
        // composites: one wave per workgroup and one sample per iteration
        // (rays of a few samples each; measured on the 1920x1080 orbit frames
        // of the 8 GiB cube: 0.21 ms against 0.28 ms with 4 waves and 2)
        MarchArgs b = a;
        b.waves = 1;
        b.unroll = 1;
        return launch_march(b, p->mode, p->filter, s);
    }
    return launch_march(a, p->mode, p->filter, s);
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" {

const char *vr_version(void) { return "vrcube 1.0 (gfx950)"; }

const char *vr_last_error(const vr_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int vr_create(vr_ctx **out, int device) {
    if (!out) return fail(nullptr, VR_EINVAL, "out is NULL");
    *out = nullptr;
    if (device == -1) {  // host-only context: argument and state checks, no launches
        vr_ctx *c = new (std::nothrow) vr_ctx();
        if (!c) return fail(nullptr, VR_ENOMEM, "out of host memory");
        c->device = -1;
        *out = c;
        return VR_OK;
    }
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(nullptr, VR_EDEVICE, "no HIP device (%s)", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, VR_EINVAL, "device %d of %d", device, n);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, VR_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    vr_ctx *c = new (std::nothrow) vr_ctx();
    if (!c) return fail(nullptr, VR_ENOMEM, "out of host memory");
    c->device = device;
#ifdef VR_DEBUG_BOUNDS
    if (hipMalloc((void **)&c->dbg, sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->dbg, 0, sizeof(uint32_t)) != hipSuccess) {
        delete c;
        return fail(nullptr, VR_EDEVICE, "debug build: cannot allocate the bounds counter");
    }
#endif
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    vr_noalloc_setup(device);
    *out = c;
    return VR_OK;
}

int vr_destroy(vr_ctx *ctx) {
    if (!ctx) return VR_OK;
    vr_stream_release(ctx);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
    if (ctx->graph_src) (void)hipGraphDestroy(ctx->graph_src);
    if (ctx->stage_pending) (void)hipEventSynchronize(ctx->stage_done);
    if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    if (ctx->dbg) (void)hipFree(ctx->dbg);
    delete ctx;
    return VR_OK;
}

int64_t vr_debug_bounds_violations(vr_ctx *ctx) {
    if (!ctx) return fail(nullptr, VR_EINVAL, "context is NULL");
#ifdef VR_DEBUG_BOUNDS
    if (ctx->device < 0 || !ctx->dbg) return fail(ctx, VR_EDEVICE, "host-only context");
    uint32_t n = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&n, ctx->dbg, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(ctx->dbg, 0, sizeof(uint32_t));
    if (e != hipSuccess) return fail(ctx, VR_EDEVICE, "bounds counter: %s", hipGetErrorString(e));
    return (int64_t)n;
#else
    return fail(ctx, VR_EUNSUPPORTED, "a release build: index-range checks need a build with VR_DEBUG_BOUNDS");
#endif
}

// ---------------------------------------------------------------------------
// volume
// ---------------------------------------------------------------------------

bool vr_layout_of(int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t B, int32_t orients, VolDev *v,
                  int64_t *bytes) {
#define layout_of vr_layout_of
    if (nx <= 0 || ny <= 0 || nz <= 0) return false;
    if (nx > (1 << 24) || ny > (1 << 24) || nz > (1 << 24)) return false;
    if (storage != VR_F32 && storage != VR_F16 && storage != VR_BF16) return false;
    if (orients != 1 && orients != 3) return false;
    VolDev d{};
    d.nx = (int32_t)nx; d.ny = (int32_t)ny; d.nz = (int32_t)nz;
    d.Bx = B > 0 ? (int32_t)std::min<int64_t>(B, nx) : (int32_t)nx;
    d.By = B > 0 ? (int32_t)std::min<int64_t>(B, ny) : (int32_t)ny;
    d.Bz = B > 0 ? (int32_t)std::min<int64_t>(B, nz) : (int32_t)nz;
    d.nbx = (int32_t)((nx + d.Bx - 1) / d.Bx);
    d.nby = (int32_t)((ny + d.By - 1) / d.By);
    d.nbz = (int32_t)((nz + d.Bz - 1) / d.Bz);
    d.Px = (d.Bx + 2 + 7) / 8 * 8; d.Py = d.By + 2; d.Pz = d.Bz + 2;
    d.brick_elems = (int64_t)d.Px * d.Py * d.Pz;
    d.dtype = storage;
    d.single = (d.nbx == 1 && d.nby == 1 && d.nbz == 1) ? 1 : 0;
    if (orients == 3 && !d.single) return false;       // copies exist for one-brick layouts only
    d.orients = orients;
    d.ori = 0;
    d.sx = 1; d.sy = d.Px; d.sz = d.Px * d.Py;
    int64_t total = d.brick_elems * d.nbx * d.nby * d.nbz;
    d.copy_off[0] = 0;
    for (int c = 1; c < orients; ++c) {
        int64_t pf, pm, ps;
        copy_pitches(d, c - 1, pf, pm, ps);
        d.copy_off[c] = d.copy_off[c - 1] + (pf * pm * ps + 127) / 128 * 128;   // 256-byte aligned copies
        copy_pitches(d, c, pf, pm, ps);
        total = d.copy_off[c] + pf * pm * ps;
    }
    if (orients == 3 && storage == VR_F32) {
        d.lpr = (int32_t)((nx + 2 + 30) / 31);
        d.line_off = (total + 127) / 128 * 128;
        total = d.line_off + (int64_t)d.Pz * d.Py * d.lpr * 32;
    }
    if (v) *v = d;
    if (bytes) *bytes = total * esize(storage);
    return true;
}

static void select_copy(VolDev &v, const CamDev &c, int32_t forced) {
    if (v.orients < 3) return;
    apply_copy(v, (forced >= 0 && forced <= 2) ? forced : best_copy(c.r));
}

int64_t vr_volume_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t brick_edge,
                        int32_t orientations) {
    int64_t b = 0;
    if (!layout_of(nx, ny, nz, storage, brick_edge, orientations, nullptr, &b)) return VR_EINVAL;
    return b;
}

int vr_describe_volume(vr_ctx *ctx, int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t brick_edge,
                       int32_t orientations, void *dst_dev, int64_t dst_bytes) {
    if (!ctx) return fail(nullptr, VR_EINVAL, "context is NULL");
    VolDev v{};
    int64_t need = 0;
    if (!layout_of(nx, ny, nz, storage, brick_edge, orientations, &v, &need))
        return fail(ctx, VR_EINVAL, "invalid cube %lldx%lldx%lld, storage %d or orientations %d (3 needs one brick)",
                    (long long)nx, (long long)ny, (long long)nz, storage, orientations);
    if (v.brick_elems >= ((int64_t)1 << 32))
        return fail(ctx, VR_EUNSUPPORTED, "a brick of %lld voxels exceeds 2^32; use a smaller brick edge",
                    (long long)v.brick_elems);
    for (int c = 1; c < v.orients; ++c) {
        int64_t pf, pm, ps;
        copy_pitches(v, c, pf, pm, ps);
        if (pf * pm * ps >= ((int64_t)1 << 32))
            return fail(ctx, VR_EUNSUPPORTED, "an orientation copy of %lld voxels exceeds 2^32", (long long)(pf * pm * ps));
    }
    if (!dst_dev) return fail(ctx, VR_EINVAL, "destination is NULL");
    if (dst_bytes < need) return fail(ctx, VR_ENOMEM, "destination holds %lld bytes, layout needs %lld",
                                      (long long)dst_bytes, (long long)need);
    v.data = dst_dev;
    v.dbg = ctx->dbg;
    vr_stream_reset(ctx);
    ctx->vol = v;
    ctx->has_volume = true;
    ctx->vol_loaded = false;
    ctx->vol_gen++;
    return ok(ctx);
}

int vr_load_slab(vr_ctx *ctx, const float *src_dev, int64_t z0, int64_t nz_slab, void *stream) {
    if (!ctx) return fail(nullptr, VR_EINVAL, "context is NULL");
    if (!ctx->has_volume) return fail(ctx, VR_ESTATE, "vr_describe_volume first");
    if (!src_dev) return fail(ctx, VR_EINVAL, "source is NULL");
    if (z0 < 0 || nz_slab <= 0 || z0 + nz_slab > ctx->vol.nz)
        return fail(ctx, VR_EINVAL, "slab [%lld, %lld) outside [0, %d)", (long long)z0, (long long)(z0 + nz_slab),
                    ctx->vol.nz);
    if (ctx->device < 0) return no_device(ctx);
    hipError_t e = launch_transcode(src_dev, ctx->vol, z0, z0 + nz_slab, (hipStream_t)stream);
    if (e != hipSuccess) return dev_check(ctx, e, "transcode");
    ctx->vol_loaded = true;
    return ok(ctx);
}

int vr_load_volume(vr_ctx *ctx, const float *src_dev, int64_t nx, int64_t ny, int64_t nz, int32_t storage,
                   int32_t brick_edge, int32_t orientations, void *dst_dev, int64_t dst_bytes, void *stream) {
    int rc = vr_describe_volume(ctx, nx, ny, nz, storage, brick_edge, orientations, dst_dev, dst_bytes);
    if (rc != VR_OK) return rc;
    return vr_load_slab(ctx, src_dev, 0, nz, stream);
}

// ---------------------------------------------------------------------------
// table, camera
// ---------------------------------------------------------------------------
int vr_set_transfer_function(vr_ctx *ctx, const float *rgba_dev, int32_t n, float vmin, float vmax) {
    if (!ctx) return fail(nullptr, VR_EINVAL, "context is NULL");
    if (!rgba_dev) return fail(ctx, VR_EINVAL, "table is NULL");
    if (n < 2 || n > 1024) return fail(ctx, VR_EINVAL, "table size %d not in [2, 1024]", n);
    if (!(vmax > vmin) || !std::isfinite(vmin) || !std::isfinite(vmax))
        return fail(ctx, VR_EINVAL, "value range [%g, %g] must have vmax > vmin", (double)vmin, (double)vmax);
    ctx->lut.rgba = (const float4 *)rgba_dev;
    ctx->lut.n = n;
    ctx->lut.vmin = vmin;
    ctx->lut.scale = (float)((double)(n - 1) / ((double)vmax - (double)vmin));
    ctx->vmax = vmax;
    ctx->has_lut = true;
    // the table's largest opacity, read back once (4 KiB at most): it bounds
    // how early a composite ray can stop, which picks the kernel (the images
    // do not depend on it).  Unknown (1) on host-only contexts or a failed
    // copy, which keeps the direct kernel for early-stopping composites.
    ctx->lut_amax = 1.0f;
    if (ctx->device >= 0) {
        std::vector<float> h((size_t)n * 4);
        if (hipMemcpy(h.data(), rgba_dev, h.size() * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess) {
            float m = 0.0f;
            for (int32_t i = 0; i < n; ++i) m = std::max(m, h[(size_t)i * 4 + 3]);
            ctx->lut_amax = std::isfinite(m) ? std::min(m, 1.0f) : 1.0f;
        } else {
            (void)hipGetLastError();
        }
    }
    return ok(ctx);
}

int vr_set_camera(vr_ctx *ctx, const vr_camera *cam) {
    if (!ctx) return fail(nullptr, VR_EINVAL, "context is NULL");
    CamDev cd{};
    int rc = check_camera(ctx, cam, &cd);
    if (rc != VR_OK) return rc;
    ctx->cam = *cam;
    ctx->camd = cd;
    ctx->has_camera = true;
    return ok(ctx);
}

// ---------------------------------------------------------------------------
// render
// ---------------------------------------------------------------------------
static int64_t ckpt_segs(const vr_ctx *ctx, const vr_render_params *p) {
    return (max_samples(ctx->vol, p->step) + vr::kCkpt - 1) / vr::kCkpt;
}

static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

int64_t vr_render_workspace_bytes(const vr_ctx *ctx, const vr_render_params *p) {
    if (!ctx || !p) return fail(ctx, VR_EINVAL, "NULL argument");
    if (!ctx->vol_loaded || !ctx->has_camera) return fail(ctx, VR_ESTATE, "volume and camera first");
    if (check_params(const_cast<vr_ctx *>(ctx), p) != VR_OK) return VR_EINVAL;
    int64_t npix = (int64_t)ctx->cam.tile_w * ctx->cam.tile_h;
    if (use_block_path(ctx, p)) return mip_blocks_workspace(npix);
    if (!p->save_for_backward) return order_bytes(ctx, p);
    return align256(npix * 4) + ckpt_segs(ctx, p) * npix * 4;
}

int vr_render(vr_ctx *ctx, const vr_render_params *p, float *out_dev, void *ws, int64_t ws_bytes, void *stream) {
    int rc = need_state(ctx, p && p->mode == VR_COMPOSITE);
    if (rc != VR_OK) return rc;
    if ((rc = check_params(ctx, p)) != VR_OK) return rc;
    if (!out_dev) return fail(ctx, VR_EINVAL, "output is NULL");
    MarchArgs a = march_args(ctx, p, ctx->camd);
    a.out = out_dev;
    if (p->save_for_backward) {
        if (p->mode != VR_COMPOSITE) return fail(ctx, VR_EUNSUPPORTED, "save_for_backward needs composite mode");
        int64_t need = vr_render_workspace_bytes(ctx, p);
        if (!ws || ws_bytes < need)
            return fail(ctx, VR_ENOMEM, "workspace %lld bytes, need %lld", (long long)ws_bytes, (long long)need);
        int64_t npix = (int64_t)ctx->cam.tile_w * ctx->cam.tile_h;
        a.taken = (int32_t *)ws;
        a.ckpt = (float *)((char *)ws + align256(npix * 4));
        a.ckpt_segs = (int32_t)ckpt_segs(ctx, p);
    }
    if (use_block_path(ctx, p)) {
        // without room for the ray records the marching kernels render the same image
        const int64_t need = mip_blocks_workspace((int64_t)ctx->cam.tile_w * ctx->cam.tile_h);
        if (ws && ws_bytes >= need) {
            MarchArgs b = a;
            b.vol = ctx->vol;                 // the x-fastest copy
            // tuning for this path: 32x16x16 blocks (42 KiB of LDS, three workgroups per CU) unless
            // lds_kib is 64..144, which takes 32x32x16 (80 KiB, two per CU); waves_per_group 8 runs
            // 512 threads on the larger blocks; slab_max blocks per run
            const vr_tuning &t = ctx->tune;
            const int32_t shape = t.waves_per_group >= 8 ? 2 : (t.lds_kib >= 64 ? 1 : 0);
            const int32_t run = t.path == 4 ? t.slab_max : 8;
            return dev_check(ctx, launch_mip_blocks(b, p->filter, ws, run, shape, (hipStream_t)stream), "render");
        }
    }
    const int64_t ob = order_bytes(ctx, p);
    void *ows = (ob > 0 && ws && ws_bytes >= ob) ? ws : nullptr;
    return dev_check(ctx, dispatch_render(ctx, a, p, (hipStream_t)stream, ows), "render");
}

int vr_render_backward(vr_ctx *ctx, const vr_render_params *p, const float *grad_out, const void *ws,
                       int64_t ws_bytes, float *grad_lut, float *grad_vol, void *stream) {
    int rc = need_state(ctx, true);
    if (rc != VR_OK) return rc;
    if ((rc = check_params(ctx, p)) != VR_OK) return rc;
    if (p->mode != VR_COMPOSITE || p->filter != VR_TRILINEAR)
        return fail(ctx, VR_EUNSUPPORTED, "gradients need composite mode with trilinear sampling");
    if (!ctx->vol.single || ctx->vol.dtype != VR_F32)
        return fail(ctx, VR_EUNSUPPORTED, "gradients need a one-brick FP32 layout");
    if (!grad_out) return fail(ctx, VR_EINVAL, "grad_out is NULL");
    vr_render_params q = *p;
    q.save_for_backward = 1;
    const int64_t need = vr_render_workspace_bytes(ctx, &q);
    if (!ws || ws_bytes < need)
        return fail(ctx, VR_ENOMEM, "workspace %lld bytes, need %lld", (long long)ws_bytes, (long long)need);
    if (!grad_lut && !grad_vol) return ok(ctx);
    MarchArgs a = march_args(ctx, &q, ctx->camd);
    const int64_t npix = (int64_t)ctx->cam.tile_w * ctx->cam.tile_h;
    a.taken = (int32_t *)ws;
    a.ckpt = (float *)((char *)ws + align256(npix * 4));
    a.ckpt_segs = (int32_t)ckpt_segs(ctx, &q);
    BackArgs b{};
    b.m = a;
    b.gout = (const float4 *)grad_out;
    b.grad_lut = grad_lut;
    b.grad_vol = grad_vol;
    return dev_check(ctx, launch_backward(b, (hipStream_t)stream), "backward");
}

int vr_count_samples(vr_ctx *ctx, const vr_render_params *p, int32_t *counts, void *stream) {
    int rc = need_state(ctx, p && p->mode == VR_COMPOSITE);
    if (rc != VR_OK) return rc;
    if ((rc = check_params(ctx, p)) != VR_OK) return rc;
    if (!counts) return fail(ctx, VR_EINVAL, "counts is NULL");
    MarchArgs a = march_args(ctx, p, ctx->camd);
    a.counts = counts;
    return dev_check(ctx, dispatch_render(ctx, a, p, (hipStream_t)stream), "count");
}

int64_t vr_touched_bitmap_bytes(const vr_ctx *ctx) {
    if (!ctx) return fail(nullptr, VR_EINVAL, "context is NULL");
    if (!ctx->has_volume) return fail(ctx, VR_ESTATE, "no volume");
    int64_t nb = (int64_t)((ctx->vol.nx + 7) / 8) * ((ctx->vol.ny + 7) / 8) * ((ctx->vol.nz + 7) / 8);
    return ((nb + 31) / 32) * 4;
}

int vr_mark_touched_blocks(vr_ctx *ctx, const vr_render_params *p, uint32_t *bitmap, int64_t bytes, void *stream) {
    int rc = need_state(ctx, p && p->mode == VR_COMPOSITE);
    if (rc != VR_OK) return rc;
    if ((rc = check_params(ctx, p)) != VR_OK) return rc;
    if (!bitmap || bytes < vr_touched_bitmap_bytes(ctx)) return fail(ctx, VR_ENOMEM, "bitmap too small");
    MarchArgs a = march_args(ctx, p, ctx->camd);
    return dev_check(ctx, launch_touch(a, p->mode, p->filter, bitmap, (hipStream_t)stream), "touch");
}

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
int vr_get_tuning(const vr_ctx *ctx, vr_tuning *out) {
    if (!ctx || !out) return fail(ctx, VR_EINVAL, "NULL argument");
    *out = ctx->tune;
    return VR_OK;
}

static bool tuning_valid(const vr_tuning &t) {
    bool shape = (t.packet_w == 8 && t.packet_h == 8) || (t.packet_w == 16 && t.packet_h == 4) ||
                 (t.packet_w == 32 && t.packet_h == 2) || (t.packet_w == 64 && t.packet_h == 1) ||
                 (t.packet_w == 4 && t.packet_h == 16);
    bool waves = t.waves_per_group == 1 || t.waves_per_group == 2 || t.waves_per_group == 4 || t.waves_per_group == 8;
    bool unroll = t.unroll == 1 || t.unroll == 2 || t.unroll == 4;
    bool pg = t.persistent_groups >= 1 && t.persistent_groups <= 32;
    bool path = t.path >= 0 && t.path <= 4;
    bool lds = t.lds_kib == 0 || (t.lds_kib >= 8 && t.lds_kib <= 144);  // 0: automatic per view
    bool slab = t.slab_max >= 1 && t.slab_max <= 64;
    // the LDS-staged kernels run 256- or 512-thread workgroups
    bool slab_shape = t.path != 2 || t.waves_per_group >= 4;
    // the compacting kernel runs workgroups of at most 256 threads (and takes
    // persistent_groups, 1..32, as packets per wave)
    bool compact_shape = t.path != 3 || t.waves_per_group <= 4;
    bool copy = t.copy >= -1 && t.copy <= 2;
    bool order = t.order >= 0 && t.order <= 3;
    return shape && waves && unroll && pg && path && lds && slab && slab_shape && compact_shape && copy && order;
}

int vr_set_tuning(vr_ctx *ctx, const vr_tuning *t) {
    if (!ctx || !t) return fail(ctx, VR_EINVAL, "NULL argument");
    if (!tuning_valid(*t)) return fail(ctx, VR_EINVAL, "invalid launch shape");
    ctx->tune = *t;
    return ok(ctx);
}

}  // extern "C"
