// vr_internal.h -- host-side launchers implemented by the kernel files and
// called by the C ABI layer (vr_api.hip).
#pragma once

#include "vr_common.h"

namespace vr {

// Transmittance checkpoints of a render saved for the adjoint: one before
// every kCkpt-th sample of a ray.  The adjoint replays kCkpt samples from a
// checkpoint into registers, so the interval is also its register budget.
constexpr int kCkptShift = 3;
constexpr int kCkpt = 1 << kCkptShift;
static_assert(kCkpt == VR_CHECKPOINT_INTERVAL, "checkpoint interval of the ABI");

struct MarchArgs {
    CamDev cam;
    VolDev vol;
    LutDev lut;
    double step;
    float thr;            // stop when T <= thr, thr = 1 - ert_alpha (ERT on)
    int32_t ert;          // early termination enabled
    void *out;            // float4 (composite) / float (MIP) per tile pixel, or NULL
    int32_t *counts;      // samples taken per pixel, or NULL
    float *ckpt;          // transmittance before samples 0, kCkpt, 2 kCkpt, ... (segment-major), or NULL
    int32_t *taken;       // samples taken per pixel (for the adjoint), or NULL
    int32_t ckpt_segs;    // checkpoints per pixel
    int32_t trans;        // 0 product, 1 log, 2 per-ray choice (log when n > 1024)
    // launch shape
    int32_t packet_w, packet_h;   // pixels per 64-lane packet
    int32_t waves;                // packets per workgroup (stacked vertically)
    int32_t groups_x;             // workgroups per tile row
    int32_t unroll;               // samples per inner iteration (direct path, one-brick layouts)
    int32_t order;                // tile order (see tile_xy)
    int32_t *tile_perm;           // order 3, LDS-staged path: workgroup -> tile, costliest first; else NULL
    uint8_t *tile_key;            // scratch of the ordering kernel: one byte per tile
};

// Bytes of caller workspace the costliest-first tile order of the LDS-staged
// path needs for a viewport of w x h pixels in bundles of bw x bh.
int64_t slab_order_bytes(int32_t w, int32_t h, int32_t bw, int32_t bh);

// K0: transcode planes [z0, z1) of a float32 (z1-z0, ny, nx) source block
// into the brick-major layout at vol.data.
hipError_t launch_transcode(const float *src, const VolDev &vol, int64_t z0, int64_t z1, hipStream_t s);

// K1/K2: single-pass render of the camera's viewport.
hipError_t launch_march(const MarchArgs &a, int32_t mode, int32_t filter, hipStream_t s);

// K1/K2, compacting form (single-brick layouts): each workgroup owns
// waves * packets_per_wave consecutive packets and its waves refill the lanes
// of finished rays from an LDS counter.  packet_w * packet_h must be 64,
// waves 1..4, packets_per_wave 1..32.
struct CompactArgs {
    MarchArgs m;
    int32_t packets;      // packets over the tile
    int32_t gxn;          // packets across the tile
    int32_t share;        // packets per workgroup
    int32_t refill_at;    // refill idle lanes once at most this many are live
};
constexpr int32_t kCompactRefillAt = 32;
hipError_t launch_march_compact(const MarchArgs &a, int32_t mode, int32_t filter, int32_t packets_per_wave,
                                hipStream_t s);

// K8: MIP in object order (single-brick layouts, x-fastest copy in a.vol):
// ray records of the tile in ws (mip_blocks_workspace bytes), blocks of the
// volume staged in LDS, one atomic maximum per (pixel, block); run = blocks
// along x per workgroup; shape 0..2 selects the block edges and threads.
int64_t mip_blocks_workspace(int64_t npix);
hipError_t launch_mip_blocks(const MarchArgs &a, int32_t filter, void *ws, int32_t run, int32_t shape,
                             hipStream_t s);

// K1/K2 with LDS-staged voxel boxes (single-brick layouts).  With
// m.order == 3 and m.tile_perm set, a first kernel orders the bundles by
// their estimated box fetch.
hipError_t launch_slab(const MarchArgs &m, int32_t mode, int32_t filter, int32_t bw, int32_t bh, int32_t cap_floats,
                       int32_t lmax, hipStream_t s);

// K7: mark touched 8^3 blocks.
hipError_t launch_touch(const MarchArgs &a, int32_t mode, int32_t filter, uint32_t *bitmap, hipStream_t s);

// K3: per-brick partials.  The table (device) holds one BrickJob per partial.
struct BrickJob {
    float *data;          // partial image (w*h*4 or w*h)
    const void *brick;    // the brick's block, or NULL: its place in the resident layout
    int32_t x0, y0, w, h; // footprint (tile-local)
    int32_t bx, by, bz;   // brick cell
    int32_t tiles_x;      // 16x16 pixel tiles across the footprint
    int32_t tile_begin;   // first tile index of this job in the flattened launch
    int32_t pad;
};
hipError_t launch_bricks(const MarchArgs &a, int32_t mode, int32_t filter, const BrickJob *jobs_dev,
                         int32_t n_jobs, int32_t total_tiles, hipStream_t s);
// K3 with LDS-staged voxel boxes (the bundle kernel's slabs inside each brick);
// the same partials as launch_bricks.
hipError_t launch_bricks_slab(const MarchArgs &m, int32_t mode, int32_t filter, const BrickJob *jobs_dev,
                              int32_t n_jobs, int32_t total_tiles, int32_t cap_floats, int32_t lmax, hipStream_t s);

// K4: composite partials (rectangles in visibility order) into the image.
struct PartRect {
    const float *data;
    int32_t x0, y0, w, h;
};
hipError_t launch_composite(const PartRect *rects_dev, int32_t n, int32_t mode, float *out,
                            int32_t tile_w, int32_t tile_h, hipStream_t s);

// K5: adjoint.
struct BackArgs {
    MarchArgs m;
    const float4 *gout;
    float *grad_lut;      // n*4 or NULL
    float *grad_vol;      // (nz,ny,nx) or NULL
};
hipError_t launch_backward(const BackArgs &a, hipStream_t s);

// K6: persistent batch.  Work items are bw x bh pixel bundles of any view.
struct ViewDev {
    CamDev cam;
    void *out;
    int32_t lut_index;
    int32_t tiles_x;      // bundles across the view
    int32_t tile_begin;   // first work item of the view
    int32_t ori;          // orientation copy the view reads
    const void *vdata;    // that copy's element 0 and element strides (resolved on the host,
    int32_t vsx, vsy, vsz;//   so the kernels select no structure field at run time)
};
struct BatchArgs {
    VolDev vol;           // copy 0 of a one-brick layout
    const ViewDev *views;
    int32_t n_views;
    int32_t total_items;
    const float4 *luts;
    int32_t lut_n;
    float vmin, scale;
    double step;
    float thr;
    int32_t ert;
    int32_t trans;
    uint32_t *queue;      // work-queue counter (zeroed by a kernel before each launch)
    int32_t bw, bh;       // bundle
    int32_t cap, lmax;    // LDS box budget (floats), thickest slab
};
hipError_t launch_batch(const BatchArgs &a, int32_t mode, int32_t filter, int32_t groups, hipStream_t s);
hipError_t launch_batch_direct(const BatchArgs &a, int32_t mode, int32_t filter, int32_t unroll, int32_t groups,
                               hipStream_t s);
hipError_t launch_reset_u32(uint32_t *p, int32_t n, hipStream_t s);

// K9: per-pixel depth of the render (one-brick layouts).
hipError_t launch_depth(const MarchArgs &a, int32_t mode, int32_t filter, float level, float *depth, hipStream_t s);
// K10: wireframe boxes over a premultiplied RGBA tile, depth-tested.
hipError_t launch_overlay(const CamDev &cam, const vr_box *boxes, int32_t n, double hw, double near,
                          const float *depth, float *img, hipStream_t s);

}  // namespace vr
