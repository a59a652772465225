// vr_api_bricks.hip -- host side of the brick path: screen footprints of the
// bricks, the partial pool layout, the visibility order and the composite
// table.  Small device tables go through the context's pinned staging area.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "vr_ctx.h"

using namespace vr;

namespace {

struct Foot {
    int32_t bx, by, bz;
    int32_t x0, y0, w, h;   // tile-local footprint
};

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Footprint of every brick in the current viewport: the bounding rectangle
// (widened by one pixel) of the projected brick corners.  A brick with a
// corner at or behind the eye plane gets the whole viewport.
std::vector<Foot> footprints(const vr_ctx *ctx) {
    const VolDev &v = ctx->vol;
    const CamDev &c = ctx->camd;
    std::vector<Foot> out;
    const int32_t tx0 = c.tile_x0, ty0 = c.tile_y0, tw = c.tile_w, th = c.tile_h;
    for (int32_t bz = 0; bz < v.nbz; ++bz)
        for (int32_t by = 0; by < v.nby; ++by)
            for (int32_t bx = 0; bx < v.nbx; ++bx) {
                double lo[3] = {(double)bx * v.Bx, (double)by * v.By, (double)bz * v.Bz};
                double hi[3] = {std::min(lo[0] + v.Bx, (double)v.nx), std::min(lo[1] + v.By, (double)v.ny),
                                std::min(lo[2] + v.Bz, (double)v.nz)};
                double cmin = 1e300, cmax = -1e300, rmin = 1e300, rmax = -1e300;
                bool whole = false;
                for (int k = 0; k < 8; ++k) {
                    double P[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
                    double d[3] = {P[0] - c.eye[0], P[1] - c.eye[1], P[2] - c.eye[2]};
                    double z = d[0] * c.f[0] + d[1] * c.f[1] + d[2] * c.f[2];
                    double x = d[0] * c.r[0] + d[1] * c.r[1] + d[2] * c.r[2];
                    double y = d[0] * c.u[0] + d[1] * c.u[1] + d[2] * c.u[2];
                    if (c.kind == VR_PERSPECTIVE) {
                        if (z <= 1e-9) { whole = true; break; }
                        x /= z;
                        y /= z;
                    }
                    double col = (x / c.a + 1.0) * c.W * 0.5 - 0.5;
                    double row = (1.0 - y / c.b) * c.H * 0.5 - 0.5;
                    cmin = std::min(cmin, col); cmax = std::max(cmax, col);
                    rmin = std::min(rmin, row); rmax = std::max(rmax, row);
                }
                int64_t x0, x1, y0, y1;   // full-frame pixel range, inclusive
                if (whole) {
                    x0 = tx0; x1 = tx0 + tw - 1; y0 = ty0; y1 = ty0 + th - 1;
                } else {
                    x0 = (int64_t)std::floor(std::max(cmin, -1e12)) - 1;
                    x1 = (int64_t)std::ceil(std::min(cmax, 1e12)) + 1;
                    y0 = (int64_t)std::floor(std::max(rmin, -1e12)) - 1;
                    y1 = (int64_t)std::ceil(std::min(rmax, 1e12)) + 1;
                    x0 = std::max<int64_t>(x0, tx0); x1 = std::min<int64_t>(x1, tx0 + tw - 1);
                    y0 = std::max<int64_t>(y0, ty0); y1 = std::min<int64_t>(y1, ty0 + th - 1);
                }
                if (x1 < x0 || y1 < y0) continue;
                out.push_back({bx, by, bz, (int32_t)(x0 - tx0), (int32_t)(y0 - ty0), (int32_t)(x1 - x0 + 1),
                               (int32_t)(y1 - y0 + 1)});
            }
    return out;
}

int chans(const vr_render_params *p) { return p->mode == VR_MIP ? 1 : 4; }

// K3: direct gathers (tuning path 1) or LDS-staged boxes (otherwise).
hipError_t launch_k3(const vr_ctx *ctx, const MarchArgs &a, const vr_render_params *p, const BrickJob *jobs,
                     int32_t n, int32_t tiles, hipStream_t s) {
    if (ctx->tune.path == 1) return launch_bricks(a, p->mode, p->filter, jobs, n, tiles, s);
    const int32_t kib = (ctx->tune.lds_kib > 0 && ctx->tune.lds_kib <= 144) ? ctx->tune.lds_kib : 64;
    return launch_bricks_slab(a, p->mode, p->filter, jobs, n, tiles, kib * 1024 / 4, ctx->tune.slab_max, s);
}

// The brick jobs of one vr_render_bricks call on a streamed volume (jobs in
// brick-id order, in the pinned staging area, their table not yet copied).
// Plan on the host which cache slot serves each brick: the bricks already
// cached first, then the others in order, each taking the least recently
// used slot.  Then enqueue: per missing brick, on the copy stream, wait
// until the last render that read its slot has finished, copy it from host
// memory into the slot and mark it ready; on the render stream, wait for it
// and launch K3 for that brick's job alone, then mark the slot free again.
// Copies of later bricks thus overlap the rendering of earlier ones.
int render_streamed(vr_ctx *ctx, const vr_render_params *p, const MarchArgs &a, BrickJob *jobs, int32_t n,
                    void *pool, size_t tbytes, hipStream_t s) {
    vr_stream_state &st = ctx->st;
    const VolDev &v = ctx->vol;
    std::vector<int64_t> id(n);
    for (int32_t i = 0; i < n; ++i) id[i] = ((int64_t)jobs[i].bz * v.nby + jobs[i].by) * v.nbx + jobs[i].bx;
    // processing order: hits, then misses (each in brick-id order)
    std::vector<int32_t> order;
    std::vector<int32_t> slot_of(n, -1);
    std::vector<char> miss(n, 0);
    for (int pass = 0; pass < 2; ++pass)
        for (int32_t i = 0; i < n; ++i) {
            if (slot_of[i] >= 0) continue;    // taken as a hit (its slot may since have been reused)
            int32_t hit = -1;
            for (int32_t k = 0; k < st.slots; ++k)
                if (st.slot_brick[k] == id[i]) { hit = k; break; }
            if ((hit >= 0) != (pass == 0)) continue;
            int32_t k = hit;
            if (k < 0) {
                k = 0;
                for (int32_t q = 1; q < st.slots; ++q)
                    if (st.slot_stamp[q] < st.slot_stamp[k]) k = q;
                st.slot_brick[k] = id[i];
                miss[i] = 1;
            }
            st.slot_stamp[k] = ++st.clock;
            slot_of[i] = k;
            order.push_back(i);
        }
    for (int32_t i = 0; i < n; ++i) {
        jobs[i].brick = st.cache + (int64_t)slot_of[i] * st.brick_bytes;
        jobs[i].tile_begin = 0;           // each job is launched alone
    }
    hipError_t e = vr_stage_copy(ctx, pool, tbytes, s);
    if (e != hipSuccess) return vr_dev_check(ctx, e, "brick table copy");
    const BrickJob *dev = (const BrickJob *)pool;
    for (int32_t i : order) {
        const int32_t k = slot_of[i];
        if (miss[i]) {
            if (st.slot_used[k] && (e = hipStreamWaitEvent(st.copy, st.slot_free[k], 0)) != hipSuccess) break;
            if ((e = hipMemcpyAsync(st.cache + (int64_t)k * st.brick_bytes, st.host + id[i] * st.brick_bytes,
                                    (size_t)st.brick_bytes, hipMemcpyHostToDevice, st.copy)) != hipSuccess)
                break;
            if ((e = hipEventRecord(st.slot_ready[k], st.copy)) != hipSuccess) break;
            if ((e = hipStreamWaitEvent(s, st.slot_ready[k], 0)) != hipSuccess) break;
            st.copied++;
        } else {
            // filled by an earlier call, possibly on another stream: order after that copy
            if ((e = hipStreamWaitEvent(s, st.slot_ready[k], 0)) != hipSuccess) break;
            st.hits++;
        }
        const int32_t tiles = jobs[i].tiles_x * ((jobs[i].h + 15) / 16);
        if ((e = launch_k3(ctx, a, p, dev + i, 1, tiles, s)) != hipSuccess) break;
        if ((e = hipEventRecord(st.slot_free[k], s)) != hipSuccess) break;
        st.slot_used[k] = 1;
    }
    if (e != hipSuccess) {
        // the slots' contents are unknown after a failed enqueue: forget them
        std::fill(st.slot_brick.begin(), st.slot_brick.end(), -1);
        return vr_dev_check(ctx, e, "streamed bricks");
    }
    return vr_dev_check(ctx, hipSuccess, "streamed bricks");
}

}  // namespace

extern "C" {

int64_t vr_bricks_pool_bytes(const vr_ctx *ctx, const vr_render_params *p) {
    if (!ctx || !p) return vr_fail(ctx, VR_EINVAL, "NULL argument");
    if (!ctx->vol_loaded || !ctx->has_camera) return vr_fail(ctx, VR_ESTATE, "volume and camera first");
    if (vr_check_params(const_cast<vr_ctx *>(ctx), p) != VR_OK) return VR_EINVAL;
    std::vector<Foot> f = footprints(ctx);
    int64_t b = align256((int64_t)f.size() * (int64_t)sizeof(BrickJob));
    for (const Foot &x : f) b += align256((int64_t)x.w * x.h * chans(p) * 4);
    return b;
}

int vr_render_bricks(vr_ctx *ctx, const vr_render_params *p, vr_partial *parts, int32_t max_parts, int32_t *n_parts,
                     void *pool, int64_t pool_bytes, void *stream) {
    int rc = vr_need_state(ctx, p && p->mode == VR_COMPOSITE, true);
    if (rc != VR_OK) return rc;
    if ((rc = vr_check_params(ctx, p)) != VR_OK) return rc;
    if (!n_parts) return vr_fail(ctx, VR_EINVAL, "n_parts is NULL");
    std::vector<Foot> f = footprints(ctx);
    *n_parts = (int32_t)f.size();
    if ((int64_t)f.size() > max_parts || (!parts && !f.empty()))
        return vr_fail(ctx, VR_ENOMEM, "%zu partials, capacity %d", f.size(), max_parts);
    const int64_t need = vr_bricks_pool_bytes(ctx, p);
    if (!pool || pool_bytes < need)
        return vr_fail(ctx, VR_ENOMEM, "pool %lld bytes, need %lld", (long long)pool_bytes, (long long)need);
    if (f.empty()) return VR_OK;
    // table + partials
    const int64_t tbytes = (int64_t)f.size() * (int64_t)sizeof(BrickJob);
    BrickJob *stage = (BrickJob *)vr_stage(ctx, (size_t)tbytes);
    if (!stage) return vr_fail(ctx, VR_EDEVICE, "pinned staging allocation failed");
    int64_t off = align256(tbytes);
    int32_t tiles = 0;
    for (size_t i = 0; i < f.size(); ++i) {
        const Foot &x = f[i];
        BrickJob &j = stage[i];
        j.data = (float *)((char *)pool + off);
        j.brick = nullptr;
        j.x0 = x.x0; j.y0 = x.y0; j.w = x.w; j.h = x.h;
        j.bx = x.bx; j.by = x.by; j.bz = x.bz;
        j.tiles_x = (x.w + 15) / 16;
        j.tile_begin = tiles;
        j.pad = 0;
        tiles += j.tiles_x * ((x.h + 15) / 16);
        parts[i].data = j.data;
        parts[i].x0 = x.x0; parts[i].y0 = x.y0; parts[i].w = x.w; parts[i].h = x.h;
        parts[i].brick_id = (x.bz * ctx->vol.nby + x.by) * ctx->vol.nbx + x.bx;
        parts[i].pad = 0;
        off += align256((int64_t)x.w * x.h * chans(p) * 4);
    }
    hipStream_t s = (hipStream_t)stream;
    MarchArgs a = vr_march_args(ctx, p, ctx->camd);
    a.vol = ctx->vol;   // partials read the x-fastest bricks
    if (ctx->st.on) return render_streamed(ctx, p, a, stage, (int32_t)f.size(), pool, (size_t)tbytes, s);
    hipError_t e = vr_stage_copy(ctx, pool, (size_t)tbytes, s);
    if (e != hipSuccess) return vr_dev_check(ctx, e, "brick table copy");
    return vr_dev_check(ctx, launch_k3(ctx, a, p, (const BrickJob *)pool, (int32_t)f.size(), tiles, s), "bricks");
}

int vr_brick_order(const vr_ctx *ctx, const vr_partial *parts, int32_t n, int32_t *order) {
    if (!ctx || (n > 0 && (!parts || !order))) return vr_fail(ctx, VR_EINVAL, "NULL argument");
    if (n < 0) return vr_fail(ctx, VR_EINVAL, "n < 0");
    if (!ctx->has_volume || !ctx->has_camera) return vr_fail(ctx, VR_ESTATE, "volume and camera first");
    const VolDev &v = ctx->vol;
    const CamDev &c = ctx->camd;
    std::vector<int64_t> key(n);
    const int64_t B[3] = {v.Bx, v.By, v.Bz};
    for (int32_t i = 0; i < n; ++i) {
        const int64_t id = parts[i].brick_id;
        if (id < 0 || id >= (int64_t)v.nbx * v.nby * v.nbz) return vr_fail(ctx, VR_EINVAL, "brick id %lld", (long long)id);
        const int64_t b[3] = {id % v.nbx, (id / v.nbx) % v.nby, id / ((int64_t)v.nbx * v.nby)};
        int64_t k = 0;
        for (int a = 0; a < 3; ++a) {
            if (c.kind == VR_PERSPECTIVE) k += std::llabs(b[a] - (int64_t)std::floor(c.eye[a] / (double)B[a]));
            else k += (c.f[a] > 0 ? 1 : (c.f[a] < 0 ? -1 : 0)) * b[a];
        }
        key[i] = k;
    }
    std::iota(order, order + n, 0);
    std::sort(order, order + n, [&](int32_t x, int32_t y) {
        return key[x] != key[y] ? key[x] < key[y] : parts[x].brick_id < parts[y].brick_id;
    });
    return VR_OK;
}

int64_t vr_composite_workspace_bytes(int32_t n) {
    if (n < 0) return VR_EINVAL;
    return align256((int64_t)n * (int64_t)sizeof(PartRect));
}

int vr_composite_bricks(vr_ctx *ctx, const vr_render_params *p, const vr_partial *parts, const int32_t *order, int32_t n,
                        float *out, void *ws, int64_t ws_bytes, void *stream) {
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    if (ctx->device < 0) return vr_fail(ctx, VR_EDEVICE, "context was created without a device");
    if (!ctx->has_camera) return vr_fail(ctx, VR_ESTATE, "no camera set");
    int rc = vr_check_params(ctx, p);
    if (rc != VR_OK) return rc;
    if (n < 0 || (n > 0 && (!parts || !order))) return vr_fail(ctx, VR_EINVAL, "bad partial list");
    if (!out) return vr_fail(ctx, VR_EINVAL, "output is NULL");
    if (n > 0 && (!ws || ws_bytes < vr_composite_workspace_bytes(n)))
        return vr_fail(ctx, VR_ENOMEM, "workspace too small");
    const int32_t tw = ctx->cam.tile_w, th = ctx->cam.tile_h;
    hipStream_t s = (hipStream_t)stream;
    if (n > 0) {
        PartRect *stage = (PartRect *)vr_stage(ctx, (size_t)n * sizeof(PartRect));
        if (!stage) return vr_fail(ctx, VR_EDEVICE, "pinned staging allocation failed");
        std::vector<char> seen(n, 0);
        for (int32_t i = 0; i < n; ++i) {
            const int32_t j = order[i];
            if (j < 0 || j >= n || seen[j]) return vr_fail(ctx, VR_EINVAL, "order is not a permutation");
            seen[j] = 1;
            const vr_partial &q = parts[j];
            if (!q.data || q.w <= 0 || q.h <= 0 || q.x0 < 0 || q.y0 < 0 || (int64_t)q.x0 + q.w > tw ||
                (int64_t)q.y0 + q.h > th)
                return vr_fail(ctx, VR_EINVAL, "partial %d outside the viewport", j);
            stage[i] = PartRect{q.data, q.x0, q.y0, q.w, q.h};
        }
        hipError_t e = vr_stage_copy(ctx, ws, (size_t)n * sizeof(PartRect), s);
        if (e != hipSuccess) return vr_dev_check(ctx, e, "composite table copy");
    }
    return vr_dev_check(ctx, launch_composite((const PartRect *)ws, n, p->mode, out, tw, th, s), "composite");
}

}  // extern "C"
