// vr_api_batch.hip -- host side of the batched renderer (one persistent launch
// over many views, optionally replayed from a HIP graph) and of the
// autotuner (timed search over launch shapes, cached as JSON).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "vr_ctx.h"

using namespace vr;

namespace {

// Views sorted by decreasing bundle count, so the largest views are handed
// out first and small ones fill the tail.
struct Plan {
    std::vector<ViewDev> table;
    int32_t total = 0;
};

int plan_views(vr_ctx *ctx, const vr_view *views, int32_t n, int32_t n_luts, Plan &pl) {
    const int32_t bw = ctx->tune.packet_w, bh = ctx->tune.packet_h * ctx->tune.waves_per_group;
    std::vector<int32_t> order(n);
    std::vector<int64_t> tiles(n);
    for (int32_t i = 0; i < n; ++i) {
        const vr_camera &c = views[i].cam;
        CamDev cd{};
        if (c.kind != VR_ORTHO && c.kind != VR_PERSPECTIVE) return vr_fail(ctx, VR_EINVAL, "view %d: camera kind", i);
        if (c.full_w <= 0 || c.full_h <= 0 || c.tile_w <= 0 || c.tile_h <= 0 || c.tile_x0 < 0 || c.tile_y0 < 0 ||
            (int64_t)c.tile_x0 + c.tile_w > c.full_w || (int64_t)c.tile_y0 + c.tile_h > c.full_h)
            return vr_fail(ctx, VR_EINVAL, "view %d: viewport outside its frame", i);
        if (c.kind == VR_PERSPECTIVE && !(c.fovy_deg > 0 && c.fovy_deg < 180))
            return vr_fail(ctx, VR_EINVAL, "view %d: fovy", i);
        if (c.kind == VR_ORTHO && !(c.half_w > 0 && c.half_h > 0)) return vr_fail(ctx, VR_EINVAL, "view %d: extents", i);
        if (!make_cam(c, &cd)) return vr_fail(ctx, VR_EINVAL, "view %d: degenerate camera", i);
        if (!views[i].out) return vr_fail(ctx, VR_EINVAL, "view %d: output is NULL", i);
        if (views[i].lut_index < 0 || views[i].lut_index >= n_luts)
            return vr_fail(ctx, VR_EINVAL, "view %d: table index %d of %d", i, views[i].lut_index, n_luts);
        tiles[i] = (int64_t)((c.tile_w + bw - 1) / bw) * ((c.tile_h + bh - 1) / bh);
    }
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return tiles[a] > tiles[b]; });
    pl.table.resize(n);
    int64_t total = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t i = order[k];
        ViewDev &v = pl.table[k];
        v = ViewDev{};
        make_cam(views[i].cam, &v.cam);
        v.out = views[i].out;
        v.lut_index = views[i].lut_index;
        v.tiles_x = (views[i].cam.tile_w + bw - 1) / bw;
        v.tile_begin = (int32_t)total;
        v.ori = ctx->vol.orients == 3 ? (ctx->tune.copy >= 0 ? ctx->tune.copy : best_copy(v.cam.r)) : 0;
        VolDev vd = ctx->vol;
        apply_copy(vd, v.ori);
        v.vdata = vd.data;
        v.vsx = vd.sx;
        v.vsy = vd.sy;
        v.vsz = vd.sz;
        total += tiles[i];
    }
    if (total >= ((int64_t)1 << 31)) return vr_fail(ctx, VR_EINVAL, "too many pixels in one batch");
    pl.total = (int32_t)total;
    return VR_OK;
}

int64_t table_bytes(int32_t n) { return vr_align256((int64_t)n * (int64_t)sizeof(ViewDev)); }

}  // namespace

extern "C" {

int64_t vr_batch_workspace_bytes(const vr_ctx *ctx, const vr_view *views, int32_t n_views) {
    (void)views;
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    if (n_views < 0) return vr_fail(ctx, VR_EINVAL, "n_views < 0");
    return table_bytes(n_views) + 256;
}

int vr_render_batch(vr_ctx *ctx, const vr_render_params *p, const vr_view *views, int32_t n_views,
                    const float *luts, int32_t n_luts, int32_t lut_n, float vmin, float vmax, void *ws, int64_t ws_bytes,
                    int32_t use_graph, void *stream) {
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    if (ctx->device < 0) return vr_fail(ctx, VR_EDEVICE, "context was created without a device");
    if (!ctx->vol_loaded) return vr_fail(ctx, VR_ESTATE, "no volume loaded");
    int rc = vr_check_params(ctx, p);
    if (rc != VR_OK) return rc;
    if (!ctx->vol.single) return vr_fail(ctx, VR_EUNSUPPORTED, "batched rendering needs a one-brick layout");
    if (ctx->tune.waves_per_group < 4) return vr_fail(ctx, VR_EUNSUPPORTED, "batched rendering uses 4- or 8-wave groups");
    if (n_views < 0 || (n_views > 0 && !views)) return vr_fail(ctx, VR_EINVAL, "bad view list");
    if (p->mode == VR_COMPOSITE) {
        if (!luts || n_luts < 1) return vr_fail(ctx, VR_EINVAL, "tables are NULL");
        if (lut_n < 2 || lut_n > 1024) return vr_fail(ctx, VR_EINVAL, "table size %d", lut_n);
        if (!(vmax > vmin)) return vr_fail(ctx, VR_EINVAL, "vmax <= vmin");
    }
    if (n_views == 0) return VR_OK;
    const int64_t need = vr_batch_workspace_bytes(ctx, views, n_views);
    if (!ws || ws_bytes < need) return vr_fail(ctx, VR_ENOMEM, "workspace %lld bytes, need %lld", (long long)ws_bytes,
                                               (long long)need);
    Plan pl;
    if ((rc = plan_views(ctx, views, n_views, p->mode == VR_COMPOSITE ? n_luts : INT32_MAX, pl)) != VR_OK) return rc;

    BatchArgs a{};
    a.vol = ctx->vol;
    a.views = (const ViewDev *)ws;
    a.n_views = n_views;
    a.total_items = pl.total;
    a.luts = (const float4 *)luts;
    a.lut_n = p->mode == VR_COMPOSITE ? lut_n : 0;
    a.vmin = vmin;
    a.scale = p->mode == VR_COMPOSITE ? (float)((double)(lut_n - 1) / ((double)vmax - (double)vmin)) : 1.0f;
    a.step = p->step;
    a.ert = p->ert_alpha < 1.0f ? 1 : 0;
    a.thr = 1.0f - p->ert_alpha;
    a.trans = p->transmittance == VR_TRANS_PRODUCT ? 0 : (p->transmittance == VR_TRANS_LOG ? 1 : (a.ert ? 2 : 1));
    a.queue = (uint32_t *)((char *)ws + table_bytes(n_views));
    a.bw = ctx->tune.packet_w;
    a.bh = ctx->tune.packet_h * ctx->tune.waves_per_group;
    // box budget, capped so that box + spare slot + table fit the 160 KiB of
    // a CU beside the kernel's static LDS (under 1 KiB)
    int32_t kib = ctx->tune.lds_kib;
    if (kib <= 0) {                                   // automatic: the widest view decides
        kib = 64;
        for (const ViewDev &v : pl.table) {
            VolDev vd = ctx->vol;
            apply_copy(vd, v.ori);
            kib = std::max(kib, vr_auto_box_kib(v.cam, vd, a.bw, a.bh));
        }
    }
    a.cap = std::min<int32_t>(kib * 1024 / 4, (160 * 1024 - 1024 - 32 - a.lut_n * 16) / 4);
    a.lmax = ctx->tune.slab_max;
    const int32_t groups = std::max(1, std::min(ctx->cus * ctx->tune.persistent_groups, pl.total));
    hipStream_t s = (hipStream_t)stream;
    // the same path rule as single renders: early-stopping composites gather
    // directly, long rays stage voxel boxes in LDS
    const int32_t direct = ctx->tune.path == 1 ||
                           (ctx->tune.path == 0 && p->mode == VR_COMPOSITE && p->ert_alpha < 1.0f);
    const int32_t unroll = ctx->tune.unroll;
    auto launch = [&](hipStream_t st) {
        return direct ? launch_batch_direct(a, p->mode, p->filter, unroll, groups, st)
                      : launch_batch(a, p->mode, p->filter, groups, st);
    };

    // view table: pinned staging -> workspace, in stream order
    void *st = vr_stage(ctx, pl.table.size() * sizeof(ViewDev));
    if (!st) return vr_fail(ctx, VR_EDEVICE, "pinned staging allocation failed");
    std::memcpy(st, pl.table.data(), pl.table.size() * sizeof(ViewDev));
    hipError_t e = vr_stage_copy(ctx, ws, pl.table.size() * sizeof(ViewDev), s);
    if (e != hipSuccess) return vr_dev_check(ctx, e, "view table copy");

    if (!use_graph) {
        e = launch_reset_u32(a.queue, 1, s);
        if (e == hipSuccess) e = launch(s);
        return vr_dev_check(ctx, e, "batch");
    }
    // graph: captured once per set of launch arguments, then replayed.  The
    // captured kernel argument holds the whole volume description (extents,
    // pitches, storage type, copies), so the key holds the volume's
    // generation: a volume described again at the same address (a caching
    // allocator may hand it out again) is captured anew.
    std::vector<int64_t> key = {(int64_t)(intptr_t)ws, (int64_t)(intptr_t)luts, (int64_t)(intptr_t)ctx->vol.data,
                                ctx->vol_gen, n_views, pl.total, lut_n, n_luts, p->mode, p->filter, a.trans, a.ert,
                                groups, a.bw, a.bh, a.cap, a.lmax, direct, unroll};
    int64_t bits;
    std::memcpy(&bits, &p->step, 8);
    key.push_back(bits);
    float fk[4] = {p->ert_alpha, vmin, vmax, 0.0f};
    for (float f : fk) {
        int32_t b32;
        std::memcpy(&b32, &f, 4);
        key.push_back(b32);
    }
    if (!ctx->graph || key != ctx->graph_key) {
        if (ctx->graph) { (void)hipGraphExecDestroy(ctx->graph); ctx->graph = nullptr; }
        if (ctx->graph_src) { (void)hipGraphDestroy(ctx->graph_src); ctx->graph_src = nullptr; }
        if (!ctx->capture_stream) {
            e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return vr_dev_check(ctx, e, "capture stream");
        }
        e = hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return vr_dev_check(ctx, e, "begin capture");
        hipError_t e1 = launch_reset_u32(a.queue, 1, ctx->capture_stream);
        hipError_t e2 = e1 == hipSuccess ? launch(ctx->capture_stream) : e1;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->capture_stream, &g);
        if (e2 != hipSuccess) { if (g) (void)hipGraphDestroy(g); return vr_dev_check(ctx, e2, "capture launch"); }
        if (e != hipSuccess) return vr_dev_check(ctx, e, "end capture");
        e = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(g); return vr_dev_check(ctx, e, "graph instantiate"); }
        ctx->graph_src = g;
        ctx->graph_key = key;
        ctx->graph_captures++;
    }
    return vr_dev_check(ctx, hipGraphLaunch(ctx->graph, s), "graph launch");
}

int vr_batch_graph_captures(const vr_ctx *ctx) { return ctx ? ctx->graph_captures : VR_EINVAL; }

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
static std::string tune_key(const vr_ctx *ctx, const vr_render_params *p, int64_t pixels, const char *what) {
    // output-size bucket: powers of two of the pixel count
    int bucket = 0;
    while (((int64_t)1 << (bucket + 1)) <= pixels) ++bucket;
    char b[256];
    snprintf(b, sizeof b, "gfx950|%s|dt%d|%dx%dx%d|b%d|o%d|m%d|f%d|e%d", what, ctx->vol.dtype, ctx->vol.nx, ctx->vol.ny,
             ctx->vol.nz, ctx->vol.single ? 0 : ctx->vol.Bx, ctx->vol.orients, p->mode, p->filter, bucket);
    return b;
}

// One-line JSON map {"key": [packet_w, packet_h, waves, unroll, groups, path, lds_kib, slab_max, copy], ...}
static bool cache_get(const char *path, const std::string &key, vr_tuning *t) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    std::string txt = ss.str();
    std::string pat = "\"" + key + "\": [";
    size_t at = txt.find(pat);
    if (at == std::string::npos) return false;
    int v[10];
    if (sscanf(txt.c_str() + at + pat.size(), "%d, %d, %d, %d, %d, %d, %d, %d, %d, %d", &v[0], &v[1], &v[2], &v[3],
               &v[4], &v[5], &v[6], &v[7], &v[8], &v[9]) != 10)
        return false;
    *t = vr_tuning{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9]};
    return true;
}

static void cache_put(const char *path, const std::string &key, const vr_tuning &t) {
    if (!path) return;
    std::vector<std::pair<std::string, std::string>> entries;
    std::ifstream f(path);
    if (f) {
        std::stringstream ss;
        ss << f.rdbuf();
        std::string txt = ss.str();
        size_t pos = 0;
        while ((pos = txt.find('"', pos)) != std::string::npos) {
            size_t e = txt.find('"', pos + 1);
            size_t lb = txt.find('[', e), rb = txt.find(']', e);
            if (e == std::string::npos || lb == std::string::npos || rb == std::string::npos) break;
            std::string k = txt.substr(pos + 1, e - pos - 1);
            if (k != key) entries.emplace_back(k, txt.substr(lb, rb - lb + 1));
            pos = rb + 1;
        }
    }
    char b[128];
    snprintf(b, sizeof b, "[%d, %d, %d, %d, %d, %d, %d, %d, %d, %d]", t.packet_w, t.packet_h, t.waves_per_group,
             t.unroll, t.persistent_groups, t.path, t.lds_kib, t.slab_max, t.copy, t.order);
    entries.emplace_back(key, b);
    std::string tmp = std::string(path) + ".tmp";
    std::ofstream o(tmp);
    o << "{";
    for (size_t i = 0; i < entries.size(); ++i)
        o << (i ? ", " : "") << "\"" << entries[i].first << "\": " << entries[i].second;
    o << "}\n";
    o.close();
    std::rename(tmp.c_str(), path);
}

// Time fn() (median of 3 after one warm-up) on stream s, in milliseconds.
template <typename F>
static float time_ms(F fn, hipStream_t s, int &rc) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) { rc = VR_EDEVICE; return 1e30f; }
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); rc = VR_EDEVICE; return 1e30f; }
    rc = fn();
    std::vector<float> t;
    for (int i = 0; i < 3 && rc == VR_OK; ++i) {
        (void)hipEventRecord(a, s);
        rc = fn();
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != VR_OK || t.empty()) return 1e30f;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

static std::vector<vr_tuning> candidates(const vr_ctx *ctx, bool batch) {
    std::vector<vr_tuning> c;
    const int shapes[3][2] = {{16, 4}, {64, 1}, {8, 8}};
    for (auto &sh : shapes) {
        for (int u : {1, 2, 4}) {
            if (batch) {
                for (int pg : {1, 2, 4}) c.push_back(vr_tuning{sh[0], sh[1], 4, u, pg, 1, 0, 16, -1, 1});
            } else {
                for (int o : {0, 1, 2}) c.push_back(vr_tuning{sh[0], sh[1], 4, u, 4, 1, 0, 16, -1, o});
                if (ctx->vol.single && u > 1)
                    for (int ppw : {1, 2}) c.push_back(vr_tuning{sh[0], sh[1], 4, u, ppw, 3, 0, 16, -1, 1});
            }
        }
        if (ctx->vol.single) {
            for (int kib : {0, 48, 64, 96, 144})
                for (int L : {8, 16, 32})
                    for (int pg : batch ? std::vector<int>{1, 2, 4} : std::vector<int>{4})
                        c.push_back(vr_tuning{sh[0], sh[1], 4, 1, pg, 2, kib, L, -1, batch ? 1 : 3});
        }
    }
    return c;
}

extern "C" {

int vr_autotune(vr_ctx *ctx, const vr_render_params *p, float *out, void *ws, int64_t ws_bytes, const char *cache_path,
                void *stream) {
    int rc = vr_need_state(ctx, p && p->mode == VR_COMPOSITE);
    if (rc != VR_OK) return rc;
    if ((rc = vr_check_params(ctx, p)) != VR_OK) return rc;
    if (!out) return vr_fail(ctx, VR_EINVAL, "output is NULL");
    const std::string key = tune_key(ctx, p, (int64_t)ctx->cam.tile_w * ctx->cam.tile_h, "render");
    vr_tuning t{};
    if (cache_get(cache_path, key, &t)) {
        ctx->tune = t;
        return VR_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const vr_tuning keep = ctx->tune;
    float best = 1e30f;
    vr_tuning best_t = keep;
    for (const vr_tuning &c : candidates(ctx, false)) {
        ctx->tune = c;
        int r2 = VR_OK;
        float ms = time_ms([&]() { return vr_render(ctx, p, out, ws, ws_bytes, stream); }, s, r2);
        if (r2 == VR_OK && ms < best) { best = ms; best_t = c; }
    }
    ctx->tune = best_t;
    if (best >= 1e29f) { ctx->tune = keep; return vr_fail(ctx, VR_EDEVICE, "no candidate launch shape ran"); }
    cache_put(cache_path, key, best_t);
    return VR_OK;
}

int vr_autotune_batch(vr_ctx *ctx, const vr_render_params *p, const vr_view *views, int32_t n_views, const float *luts,
                      int32_t n_luts, int32_t lut_n, float vmin, float vmax, void *ws, int64_t ws_bytes,
                      const char *cache_path, void *stream) {
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    if (!ctx->vol_loaded) return vr_fail(ctx, VR_ESTATE, "no volume loaded");
    int rc = vr_check_params(ctx, p);
    if (rc != VR_OK) return rc;
    if (n_views <= 0 || !views) return vr_fail(ctx, VR_EINVAL, "no views");
    int64_t px = 0;
    for (int32_t i = 0; i < n_views; ++i) px += (int64_t)views[i].cam.tile_w * views[i].cam.tile_h;
    const std::string key = tune_key(ctx, p, px, "batch");
    vr_tuning t{};
    if (cache_get(cache_path, key, &t)) {
        ctx->tune = t;
        return VR_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const vr_tuning keep = ctx->tune;
    float best = 1e30f;
    vr_tuning best_t = keep;
    for (const vr_tuning &c : candidates(ctx, true)) {
        ctx->tune = c;
        int r2 = VR_OK;
        float ms = time_ms([&]() {
            return vr_render_batch(ctx, p, views, n_views, luts, n_luts, lut_n, vmin, vmax, ws, ws_bytes, 0, stream);
        }, s, r2);
        if (r2 == VR_OK && ms < best) { best = ms; best_t = c; }
    }
    ctx->tune = best_t;
    if (best >= 1e29f) { ctx->tune = keep; return vr_fail(ctx, VR_EDEVICE, "no candidate launch shape ran"); }
    cache_put(cache_path, key, best_t);
    return VR_OK;
}

}  // extern "C"
