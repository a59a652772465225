// vr_ctx.h -- the context object behind vr_ctx* and the helpers the C ABI
// files share (error reporting, state and argument checks, staging).
#pragma once

#include <string>
#include <vector>

#include "vr_internal.h"

// Out-of-core bricks: the packed bricks stay in (pinned) host memory and a
// device cache of `slots` bricks holds the ones being rendered, filled on a
// copy stream of the context's own and evicted least recently used first.
struct vr_stream_state {
    bool on = false;
    const uint8_t *host = nullptr;
    int64_t host_bytes = 0;
    uint8_t *cache = nullptr;
    int32_t slots = 0;
    int64_t brick_bytes = 0;
    std::vector<int64_t> slot_brick;   // brick held by each slot, -1 empty
    std::vector<int64_t> slot_stamp;   // last use (for LRU)
    std::vector<char> slot_used;       // slot_free has been recorded at least once
    std::vector<hipEvent_t> slot_free; // recorded after the last render that read the slot
    std::vector<hipEvent_t> slot_ready;// recorded after the copy into the slot
    int64_t clock = 0, copied = 0, hits = 0;
    hipStream_t copy = nullptr;
};

struct vr_ctx {
    int device = 0;       // -1: host-only context (checks, no launches)
    std::string err;
    // volume
    bool has_volume = false;
    vr::VolDev vol{};
    bool vol_loaded = false;
    int64_t vol_gen = 0;  // bumped by every vr_describe_volume: part of the batch graph's key
    // table
    bool has_lut = false;
    vr::LutDev lut{};
    float vmax = 1.0f;
    float lut_amax = 1.0f;   // largest opacity of the table (kernel choice only)
    // camera
    bool has_camera = false;
    vr_camera cam{};
    vr::CamDev camd{};
    // launch shape
    vr_tuning tune{16, 4, 4, 2, 4, 0, 0, 16, -1, 3};
    // pinned staging for small device tables, and the event of its last copy
    void *stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr;
    bool stage_pending = false;
    // batch graph cache: the captured (queue reset + persistent kernel) pair
    // and the launch arguments it was captured with
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_src = nullptr;
    std::vector<int64_t> graph_key;
    hipStream_t capture_stream = nullptr;
    int32_t cus = 256;    // compute units of the device
    uint32_t *dbg = nullptr;   // debug builds: the index-range violation counter (device memory)
    int32_t graph_captures = 0;
    vr_stream_state st;   // out-of-core bricks (off unless vr_describe_streamed_volume)
};

int vr_fail(const vr_ctx *ctx, int code, const char *fmt, ...);
int vr_dev_check(vr_ctx *ctx, hipError_t e, const char *what);
int vr_check_params(vr_ctx *ctx, const vr_render_params *p);
int vr_need_state(vr_ctx *ctx, bool lut_needed, bool streamed_ok = false);
// Layout of a cube (one brick or many, 1 or 3 orientation copies): false if
// invalid; *v and *bytes (either may be NULL) describe it.
extern "C" bool vr_layout_of(int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t B, int32_t orients,
                             vr::VolDev *v, int64_t *bytes);
// Streamed volumes: drop the cache bookkeeping (the volume is described
// again), and release the copy stream and events (context destroyed).
void vr_stream_reset(vr_ctx *ctx);
void vr_stream_release(vr_ctx *ctx);
vr::MarchArgs vr_march_args(vr_ctx *ctx, const vr_render_params *p, const vr::CamDev &cam);
int32_t vr_auto_box_kib(const vr::CamDev &c, const vr::VolDev &v, int32_t bw, int32_t bh);
// The estimate behind it: KiB of the widest far-side box at slab thickness 2.
double vr_box_estimate_kib(const vr::CamDev &c, const vr::VolDev &v, int32_t bw, int32_t bh);
// Pinned host staging of at least `bytes`; waits for the previous copy out of
// it first.  NULL on failure.
void *vr_stage(vr_ctx *ctx, size_t bytes);
// Copy the first `bytes` of the staging area to dst on stream s and record
// the copy's completion.
hipError_t vr_stage_copy(vr_ctx *ctx, void *dst, size_t bytes, hipStream_t s);

int64_t vr_align256(int64_t x);
// Resolve the device address of the fixed scratch array behind
// vr_render_noalloc for `device` (which the caller has made current).
void vr_noalloc_setup(int device);
