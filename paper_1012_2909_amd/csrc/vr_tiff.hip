// vr_tiff.hip -- the display pyramid's C ABI and its pyramidal tiled TIFF
// writer (section 3: a static high-resolution render is stored as TIFF and
// converted to a pyramidal tiled TIFF, the format the tiled display's image
// server reads).  The writer is host code: one IFD per pyramid level, chained
// from full resolution down, each level cut into square tiles of RGBA8 with
// associated (premultiplied) alpha, uncompressed; BigTIFF when the offsets
// would not fit 32 bits.
#include <cstdio>
#include <cstring>
#include <vector>

#include "vr_ctx.h"

namespace vr {
hipError_t launch_pyramid(const float *src, int32_t w, int32_t h, int32_t levels, uint8_t *dst, hipStream_t s);
}

namespace {

// Levels of a w x h pyramid with tiles of `tile`: halve (rounding up) until
// both sides fit one tile.
int32_t pyramid_levels(int32_t w, int32_t h, int32_t tile) {
    int32_t n = 1;
    while (w > tile || h > tile) {
        w = (w + 1) / 2;
        h = (h + 1) / 2;
        ++n;
    }
    return n;
}

int64_t pyramid_bytes(int32_t w, int32_t h, int32_t levels) {
    int64_t b = 0;
    for (int32_t l = 0; l < levels; ++l) {
        b += (int64_t)w * h * 4;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    return b;
}

struct Writer {
    FILE *f = nullptr;
    bool big = false;
    bool ok = true;
    void put(const void *p, size_t n) { ok = ok && fwrite(p, 1, n, f) == n; }
    void u16(uint16_t v) { put(&v, 2); }
    void u32(uint32_t v) { put(&v, 4); }
    void u64(uint64_t v) { put(&v, 8); }
    void off(uint64_t v) { big ? u64(v) : u32((uint32_t)v); }
    // one IFD entry whose value fits the entry (count values of `type`)
    void entry(uint16_t tag, uint16_t type, uint64_t count, uint64_t value) {
        u16(tag);
        u16(type);
        big ? u64(count) : u32((uint32_t)count);
        if (type == 3 && count == 1) {          // SHORT, left-justified in the value field
            u16((uint16_t)value);
            big ? (u16(0), u32(0)) : u16(0);
        } else {
            off(value);
        }
    }
};

}  // namespace

extern "C" {

int64_t vr_pyramid_bytes(int32_t w, int32_t h, int32_t tile, int32_t *levels_out) {
    if (w <= 0 || h <= 0 || tile < 16 || tile % 16 != 0 || tile > 4096)
        return vr_fail(nullptr, VR_EINVAL, "pyramid of %d x %d with tile %d (tile: a multiple of 16 in [16, 4096])",
                       w, h, tile);
    const int32_t L = pyramid_levels(w, h, tile);
    if (levels_out) *levels_out = L;
    return pyramid_bytes(w, h, L);
}

int vr_build_pyramid(vr_ctx *ctx, const float *rgba_dev, int32_t w, int32_t h, int32_t tile, uint8_t *dst_dev,
                     int64_t dst_bytes, void *stream) {
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    int32_t L = 0;
    const int64_t need = vr_pyramid_bytes(w, h, tile, &L);
    if (need < 0) return vr_fail(ctx, VR_EINVAL, "%s", vr_last_error(nullptr));
    if (!rgba_dev || !dst_dev) return vr_fail(ctx, VR_EINVAL, "NULL image or pyramid");
    if (((uintptr_t)rgba_dev & 15) || ((uintptr_t)dst_dev & 3))
        return vr_fail(ctx, VR_EINVAL, "image must be 16-byte aligned and the pyramid 4-byte aligned");
    if (dst_bytes < need) return vr_fail(ctx, VR_ENOMEM, "pyramid buffer %lld bytes, need %lld", (long long)dst_bytes,
                                         (long long)need);
    if (ctx->device < 0) return vr_fail(ctx, VR_EDEVICE, "host-only context");
    return vr_dev_check(ctx, vr::launch_pyramid(rgba_dev, w, h, L, dst_dev, (hipStream_t)stream), "pyramid");
}

int vr_write_pyramid_tiff(const char *path, const uint8_t *pyr, int32_t w, int32_t h, int32_t tile,
                          int32_t bigtiff) {
    int32_t L = 0;
    if (!path || !pyr) return vr_fail(nullptr, VR_EINVAL, "NULL path or pyramid");
    if (vr_pyramid_bytes(w, h, tile, &L) < 0) return VR_EINVAL;
    // sizes first: does every offset fit 32 bits?
    const uint64_t tile_bytes = (uint64_t)tile * tile * 4;
    uint64_t total = 16;
    {
        int32_t lw = w, lh = h;
        for (int32_t l = 0; l < L; ++l) {
            const uint64_t nt = (uint64_t)((lw + tile - 1) / tile) * ((lh + tile - 1) / tile);
            total += nt * tile_bytes + 512 + nt * 16;
            lw = (lw + 1) / 2;
            lh = (lh + 1) / 2;
        }
    }
    Writer W;
    if (bigtiff != 0 && bigtiff != 1) return vr_fail(nullptr, VR_EINVAL, "bigtiff %d not 0 or 1", bigtiff);
    W.big = bigtiff == 1 || total >= 0xFFFFFF00ull;
    W.f = std::fopen(path, "wb");
    if (!W.f) return vr_fail(nullptr, VR_EINVAL, "cannot open %s for writing", path);
    // header; the first IFD's offset is patched once known
    W.put("II", 2);
    if (W.big) { W.u16(43); W.u16(8); W.u16(0); W.u64(0); }
    else { W.u16(42); W.u32(0); }
    uint64_t link_at = W.big ? 8 : 4;            // where the previous IFD's "next" offset goes
    std::vector<uint8_t> buf(tile_bytes);
    const uint8_t *lev = pyr;
    int32_t lw = w, lh = h;
    for (int32_t l = 0; l < L && W.ok; ++l) {
        const int32_t tx = (lw + tile - 1) / tile, ty = (lh + tile - 1) / tile;
        std::vector<uint64_t> offs((size_t)tx * ty);
        for (int32_t j = 0; j < ty; ++j)
            for (int32_t i = 0; i < tx; ++i) {
                std::memset(buf.data(), 0, buf.size());
                const int32_t cw = std::min(tile, lw - i * tile), ch = std::min(tile, lh - j * tile);
                for (int32_t r = 0; r < ch; ++r)
                    std::memcpy(buf.data() + (size_t)r * tile * 4,
                                lev + ((size_t)(j * tile + r) * lw + (size_t)i * tile) * 4, (size_t)cw * 4);
                offs[(size_t)j * tx + i] = (uint64_t)std::ftell(W.f);
                W.put(buf.data(), buf.size());
            }
        // out-of-line arrays: BitsPerSample (classic only), tile offsets, byte counts
        const uint64_t bps_at = (uint64_t)std::ftell(W.f);
        if (!W.big) for (int c = 0; c < 4; ++c) W.u16(8);
        const uint64_t n = offs.size();
        const uint64_t offs_at = (uint64_t)std::ftell(W.f);
        for (uint64_t o : offs) W.off(o);
        const uint64_t cnts_at = (uint64_t)std::ftell(W.f);
        for (uint64_t k = 0; k < n; ++k) W.off(tile_bytes);
        if (std::ftell(W.f) & 1) W.put("\0", 1);  // IFDs start on a word boundary
        // the IFD
        const uint64_t ifd_at = (uint64_t)std::ftell(W.f);
        const uint16_t T_OFF = W.big ? 16 : 4;      // LONG8 / LONG
        const int n_ent = 13;
        W.big ? W.u64(n_ent) : W.u16(n_ent);
        W.entry(254, 4, 1, l == 0 ? 0 : 1);         // NewSubfileType: reduced-resolution levels
        W.entry(256, 4, 1, (uint64_t)lw);           // ImageWidth
        W.entry(257, 4, 1, (uint64_t)lh);           // ImageLength
        if (W.big) {                                // BitsPerSample 8,8,8,8 inline
            W.u16(258); W.u16(3); W.u64(4); W.u16(8); W.u16(8); W.u16(8); W.u16(8);
        } else {
            W.entry(258, 3, 4, bps_at);
        }
        W.entry(259, 3, 1, 1);                      // Compression: none
        W.entry(262, 3, 1, 2);                      // Photometric: RGB
        W.entry(277, 3, 1, 4);                      // SamplesPerPixel
        W.entry(284, 3, 1, 1);                      // PlanarConfiguration: chunky
        W.entry(322, 4, 1, (uint64_t)tile);         // TileWidth
        W.entry(323, 4, 1, (uint64_t)tile);         // TileLength
        if (n == 1) { W.entry(324, T_OFF, 1, offs[0]); W.entry(325, T_OFF, 1, tile_bytes); }
        else { W.entry(324, T_OFF, n, offs_at); W.entry(325, T_OFF, n, cnts_at); }
        W.entry(338, 3, 1, 1);                      // ExtraSamples: associated alpha
        const uint64_t next_at = (uint64_t)std::ftell(W.f);
        W.off(0);
        // link this IFD from the header or the previous IFD
        const long end = std::ftell(W.f);
        W.ok = W.ok && std::fseek(W.f, (long)link_at, SEEK_SET) == 0;
        W.off(ifd_at);
        W.ok = W.ok && std::fseek(W.f, end, SEEK_SET) == 0;
        link_at = next_at;
        lev += (size_t)lw * lh * 4;
        lw = (lw + 1) / 2;
        lh = (lh + 1) / 2;
    }
    const bool closed = std::fclose(W.f) == 0;
    if (!W.ok || !closed) return vr_fail(nullptr, VR_EINVAL, "write to %s failed", path);
    return VR_OK;
}

}  // extern "C"
