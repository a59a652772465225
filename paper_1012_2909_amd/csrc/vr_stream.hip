// vr_stream.hip -- out-of-core bricks (section 1: cubes larger than a
// machine's memory are rendered as bricks; section 3: WALLABY's expected
// 6144 x 6144 x 16384 cube): the host-side packer of the brick-major layout,
// and the description of a volume whose bricks stay in host memory and reach
// the GPU through a device cache (the streamed rendering itself is in
// vr_api_bricks.hip).
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <type_traits>
#include <vector>

#include "vr_ctx.h"

using namespace vr;

namespace {

inline uint16_t bf16_rne(float v) {
    uint32_t u;
    std::memcpy(&u, &v, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                             // nearest, ties to even
    return (uint16_t)(u >> 16);
}

inline int64_t clampi(int64_t i, int64_t hi) { return i < 0 ? 0 : (i > hi ? hi : i); }

// One brick of the layout v (x-fastest, apron clamped to the cube's faces),
// written exactly as K0 writes it on the device.
template <typename S>
void pack_brick(const float *src, const VolDev &v, int64_t b, uint8_t *dst) {
    const int64_t bx = b % v.nbx, by = (b / v.nbx) % v.nby, bz = b / ((int64_t)v.nbx * v.nby);
    S *out = (S *)dst + b * v.brick_elems;
    for (int64_t lz = 0; lz < v.Pz; ++lz) {
        const int64_t gz = clampi(bz * v.Bz - 1 + lz, v.nz - 1);
        for (int64_t ly = 0; ly < v.Py; ++ly) {
            const int64_t gy = clampi(by * v.By - 1 + ly, v.ny - 1);
            const float *srow = src + (gz * v.ny + gy) * (int64_t)v.nx;
            S *drow = out + (lz * v.Py + ly) * (int64_t)v.Px;
            for (int64_t lx = 0; lx < v.Px; ++lx) {
                const float x = srow[clampi(bx * v.Bx - 1 + lx, v.nx - 1)];
                if constexpr (sizeof(S) == 4) drow[lx] = x;
                else if constexpr (std::is_same<S, _Float16>::value) drow[lx] = (_Float16)x;
                else drow[lx] = bf16_rne(x);
            }
        }
    }
}

}  // namespace

void vr_stream_reset(vr_ctx *ctx) {
    vr_stream_state &st = ctx->st;
    st.on = false;
    st.host = nullptr;
    st.cache = nullptr;
    std::fill(st.slot_brick.begin(), st.slot_brick.end(), -1);
}

void vr_stream_release(vr_ctx *ctx) {
    vr_stream_state &st = ctx->st;
    if (st.copy) (void)hipStreamSynchronize(st.copy);
    for (hipEvent_t e : st.slot_free) if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : st.slot_ready) if (e) (void)hipEventDestroy(e);
    st.slot_free.clear();
    st.slot_ready.clear();
    if (st.copy) (void)hipStreamDestroy(st.copy);
    st.copy = nullptr;
}

extern "C" {

int64_t vr_brick_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t brick_edge) {
    VolDev v{};
    int64_t total = 0;
    if (brick_edge <= 0 || !vr_layout_of(nx, ny, nz, storage, brick_edge, 1, &v, &total)) return VR_EINVAL;
    return total / ((int64_t)v.nbx * v.nby * v.nbz);
}

int vr_pack_bricks_host(const float *src, int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t brick_edge,
                        void *dst, int64_t dst_bytes, int32_t threads) {
    VolDev v{};
    int64_t need = 0;
    if (!src || !dst) return vr_fail(nullptr, VR_EINVAL, "NULL source or destination");
    if (brick_edge <= 0 || !vr_layout_of(nx, ny, nz, storage, brick_edge, 1, &v, &need))
        return vr_fail(nullptr, VR_EINVAL, "invalid cube %lldx%lldx%lld, storage %d or brick edge %d",
                       (long long)nx, (long long)ny, (long long)nz, storage, brick_edge);
    if (dst_bytes < need)
        return vr_fail(nullptr, VR_ENOMEM, "destination holds %lld bytes, layout needs %lld", (long long)dst_bytes,
                       (long long)need);
    const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
    int32_t nt = threads > 0 ? threads : (int32_t)std::max(1u, std::thread::hardware_concurrency());
    nt = (int32_t)std::min<int64_t>(nt, nb);
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (int64_t b; (b = next.fetch_add(1)) < nb;) {
            if (storage == VR_F32) pack_brick<float>(src, v, b, (uint8_t *)dst);
            else if (storage == VR_F16) pack_brick<_Float16>(src, v, b, (uint8_t *)dst);
            else pack_brick<uint16_t>(src, v, b, (uint8_t *)dst);
        }
    };
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (std::thread &t : pool) t.join();
    return VR_OK;
}

int vr_describe_streamed_volume(vr_ctx *ctx, int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t brick_edge,
                                const void *host_bricks, int64_t host_bytes, void *cache_dev, int64_t cache_bytes) {
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    if (ctx->device < 0) return vr_fail(ctx, VR_EDEVICE, "host-only context");
    VolDev v{};
    int64_t need = 0;
    if (brick_edge <= 0 || !vr_layout_of(nx, ny, nz, storage, brick_edge, 1, &v, &need))
        return vr_fail(ctx, VR_EINVAL, "invalid cube %lldx%lldx%lld, storage %d or brick edge %d", (long long)nx,
                       (long long)ny, (long long)nz, storage, brick_edge);
    if (v.brick_elems >= ((int64_t)1 << 32))
        return vr_fail(ctx, VR_EUNSUPPORTED, "a brick of %lld voxels exceeds 2^32", (long long)v.brick_elems);
    if (!host_bricks || !cache_dev) return vr_fail(ctx, VR_EINVAL, "NULL host bricks or cache");
    if (host_bytes < need)
        return vr_fail(ctx, VR_ENOMEM, "host bricks hold %lld bytes, layout needs %lld", (long long)host_bytes,
                       (long long)need);
    const int64_t bb = need / ((int64_t)v.nbx * v.nby * v.nbz);
    const int64_t slots = cache_bytes / bb;
    if (slots < 1) return vr_fail(ctx, VR_ENOMEM, "cache of %lld bytes holds no brick of %lld", (long long)cache_bytes,
                                  (long long)bb);
    if (slots > (1 << 20)) return vr_fail(ctx, VR_EINVAL, "cache of %lld slots", (long long)slots);
    vr_stream_state &st = ctx->st;
    // the copy stream (default priority) and one pair of events per slot
    if (!st.copy && hipStreamCreateWithFlags(&st.copy, hipStreamNonBlocking) != hipSuccess)
        return vr_fail(ctx, VR_EDEVICE, "copy stream");
    if (st.copy) (void)hipStreamSynchronize(st.copy);
    while ((int64_t)st.slot_free.size() < slots) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            return vr_fail(ctx, VR_EDEVICE, "event creation");
        }
        st.slot_free.push_back(a);
        st.slot_ready.push_back(b);
    }
    v.data = cache_dev;
    v.dbg = ctx->dbg;
    ctx->vol = v;
    ctx->has_volume = true;
    ctx->vol_loaded = true;            // the bricks are packed already
    ctx->vol_gen++;
    st.on = true;
    st.host = (const uint8_t *)host_bricks;
    st.host_bytes = host_bytes;
    st.cache = (uint8_t *)cache_dev;
    st.slots = (int32_t)slots;
    st.brick_bytes = bb;
    st.slot_brick.assign((size_t)slots, -1);
    st.slot_stamp.assign((size_t)slots, 0);
    st.slot_used.assign((size_t)slots, 0);
    st.clock = st.copied = st.hits = 0;
    return VR_OK;
}

int vr_stream_stats(const vr_ctx *ctx, int64_t *bricks_copied, int64_t *cache_hits, int32_t *slots) {
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    if (!ctx->st.on) return vr_fail(ctx, VR_ESTATE, "no streamed volume");
    if (bricks_copied) *bricks_copied = ctx->st.copied;
    if (cache_hits) *cache_hits = ctx->st.hits;
    if (slots) *slots = ctx->st.slots;
    return VR_OK;
}

}  // extern "C"
