/*
 * vr.h -- C ABI of the MI355X ray caster for float32 spectral cubes.
 *
 * The library renders a 3D spectral cube (RA x Dec x frequency, float32) by
 * ray casting, the rendering method of the paper's GPU framework (abstract,
 * section 1), at a user-chosen orientation and output size, including one
 * viewport of a larger frame such as one panel of the 5x5 wall of 1920x1080
 * screens (section 3).  Rendering is separate from display (section 4): the
 * caller owns every buffer and decides what to do with the images.
 *
 * Conventions used by every call (the paper gives no formulas; these are
 * the readings the library implements):
 *  - World: voxel units.  The cube occupies [0,nx]x[0,ny]x[0,nz]; voxel
 *    (i,j,k) has its centre at (i+1/2, j+1/2, k+1/2) and is element
 *    (k*ny + j)*nx + i of a C-ordered (nz, ny, nx) float32 array.
 *  - Camera: f = unit(target-eye), r = unit(f x up), u = r x f.  Full-frame
 *    pixel (col, row) has sx = (2(col+1/2)/W - 1) a, sy = (1 - 2(row+1/2)/H) b.
 *    Perspective: a = tan(fovy/2) W/H, b = tan(fovy/2); the ray starts at
 *    eye with direction unit(f + sx r + sy u).  Orthographic: a = half_w,
 *    b = half_h; the ray starts at eye + sx r + sy u with direction f.
 *  - Clip: the ray's slab interval [tn, tf] against the cube; t0 = max(tn,0),
 *    t1 = tf; no samples when t1 <= t0.
 *  - Samples: t_k = t0 + (k + 1/2) step, for every k >= 0 with t_k < t1.
 *  - Trilinear: q = p - 1/2 clamped to [0, N-1] per axis, i = min(floor q,
 *    N-2), f = q - i (clamp-to-edge).  Nearest: clamp(floor p, 0, N-1).
 *  - Transfer function: n straight-RGBA entries over [vmin, vmax]; x =
 *    clamp((s - vmin)/(vmax - vmin), 0, 1) (n-1), j = min(floor x, n-2),
 *    w = x - j, rgba = (1-w) L[j] + w L[j+1].
 *  - Composite: front to back, C += (1-A) a c, A += (1-A) a, stopping after
 *    the sample at which A >= ert_alpha (ert_alpha >= 1: never).  Output is
 *    premultiplied RGBA (C, A) with no background.
 *  - MIP: the maximum sample value; -inf when the ray takes no sample.
 *  - Bricks: edge-B bricks partition space into half-open boxes; a sample
 *    belongs to the brick holding its position.  Each brick composites its
 *    own samples (with its own early stop); partials combine with the
 *    front-to-back "over" operator in key order: Manhattan distance of the
 *    brick cell from the eye's cell (perspective) or sum_a sign(f_a) i_a
 *    (orthographic), ties by brick id.
 *
 * Memory and streams.  Every device pointer is borrowed: the caller
 * allocates it (the Python layer uses torch tensors) and keeps it alive until
 * the stream work that uses it has finished.  The library never allocates
 * device memory; it allocates only a small pinned host staging area per
 * context (for brick tables).  Each call enqueues its kernels on the HIP
 * stream passed in (NULL = the default stream) and returns without
 * synchronising.
 *
 * Errors.  Every call returns a vr_status; argument and state checks are
 * synchronous, and vr_last_error() then holds a message.  A failed launch
 * returns VR_EDEVICE.  No call aborts or throws across the ABI.  A context is
 * used by one host thread at a time.
 */
#ifndef VR_H
#define VR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vr_ctx vr_ctx;

/* A render saved for the adjoint (save_for_backward) keeps, per pixel, the
 * transmittance in front of every VR_CHECKPOINT_INTERVAL-th sample of the
 * ray; the adjoint replays that many samples from a checkpoint. */
#define VR_CHECKPOINT_INTERVAL 8

typedef enum {
    VR_OK = 0,
    VR_EINVAL = -1,       /* bad argument */
    VR_ESTATE = -2,       /* call made in the wrong state (e.g. render before load) */
    VR_ENOMEM = -3,       /* caller's buffer or workspace too small */
    VR_EDEVICE = -4,      /* HIP error */
    VR_EUNSUPPORTED = -5  /* valid but not supported by the library */
} vr_status;

typedef enum { VR_F32 = 0, VR_F16 = 1, VR_BF16 = 2 } vr_dtype;
typedef enum { VR_COMPOSITE = 0, VR_MIP = 1 } vr_mode;
typedef enum { VR_TRILINEAR = 0, VR_NEAREST = 1 } vr_filter;
typedef enum { VR_ORTHO = 0, VR_PERSPECTIVE = 1 } vr_projection;
/* Transmittance bookkeeping of the composite: the running product T *= (1-a)
 * in FP32, or log T accumulated with a compensated sum of log1p(-a) (for long
 * rays, where the product's rounding grows with the sample count).  AUTO
 * takes the log form when early termination is off or a ray has more than
 * 1024 samples. */
typedef enum { VR_TRANS_AUTO = 0, VR_TRANS_PRODUCT = 1, VR_TRANS_LOG = 2 } vr_transmittance;

/* View.  Geometry is FP64 so that the caller's camera is used exactly. */
typedef struct {
    int32_t kind;                 /* vr_projection */
    double eye[3], target[3], up[3];
    double fovy_deg;              /* perspective: full vertical field of view, degrees, in (0, 180) */
    double half_w, half_h;        /* orthographic: half extents of the frame, world units, > 0 */
    int32_t full_w, full_h;       /* full frame in pixels (e.g. 9600 x 5400 for the 5x5 wall) */
    int32_t tile_x0, tile_y0;     /* viewport rendered by this call, inside the full frame */
    int32_t tile_w, tile_h;
} vr_camera;

typedef struct {
    int32_t mode;                 /* vr_mode */
    int32_t filter;               /* vr_filter */
    double step;                  /* sample spacing in voxels, in [1e-4, 1e6] (0.5 in every workload) */
    float ert_alpha;              /* early-termination opacity; >= 1 disables */
    int32_t transmittance;        /* vr_transmittance */
    int32_t save_for_backward;    /* composite only: write transmittance checkpoints to the workspace */
} vr_render_params;

/* One brick's partial image: a footprint rectangle of the tile (tile-local
 * pixel coordinates) holding premultiplied RGBA (h*w*4 floats, row-major)
 * or, in MIP mode, h*w maxima. */
typedef struct {
    float *data;                  /* device pointer inside the caller's pool */
    int32_t x0, y0, w, h;
    int32_t brick_id;             /* (bz*nby + by)*nbx + bx */
    int32_t pad;
} vr_partial;

/* One view of a batch. */
typedef struct {
    vr_camera cam;
    int32_t lut_index;            /* table of this view in the batch's table array */
    int32_t pad;
    void *out;                    /* device image: tile_h*tile_w*4 floats (composite) or *1 (MIP) */
} vr_view;

/* Tunable launch shape of the renderer (see vr_autotune).  A workgroup
 * renders a bundle of packet_w x (packet_h * waves_per_group) pixels, one
 * 64-lane wave per packet_w x packet_h packet. */
typedef struct {
    int32_t packet_w, packet_h;   /* pixels per wavefront packet: 8x8, 16x4, 32x2, 64x1, 4x16 */
    int32_t waves_per_group;      /* 1, 2, 4, 8 (LDS-staged path: 4 or 8); path 0 renders early-stopping
                                     composites on one-brick layouts with 1 wave and unroll 1 whatever
                                     these two fields say (the measured best for rays of a few samples) */
    int32_t unroll;               /* direct path on one-brick layouts: samples per inner iteration, 1, 2, 4 */
    int32_t persistent_groups;    /* batched launch: workgroups per CU; path 3: packets per wave in a
                                     workgroup's share; 1..32 */
    int32_t path;                 /* 0 auto, 1 direct gathers, 2 LDS-staged voxel boxes (one-brick layouts),
                                     3 direct gathers whose waves refill the lanes of finished rays with the
                                     next pixels of their workgroup's share of packets, once a ballot shows
                                     at most half of the lanes live (one-brick layouts, waves_per_group <= 4),
                                     4 MIP in object order: blocks of the volume in LDS, one atomic maximum per
                                     pixel and block (one-brick layouts, MIP only; needs the per-pixel ray
                                     records vr_render_workspace_bytes counts, else renders as path 0).
                                     Path 4 reads lds_kib 64..144 as 32x32x16 blocks (else 32x16x16),
                                     waves_per_group 8 as 512 threads on the larger blocks, slab_max as the
                                     blocks each workgroup walks along x.  Path 0 takes path 4 for MIP views
                                     oblique to the axes (lds_kib 0 and waves_per_group >= 4) */
    int32_t lds_kib;              /* LDS-staged path: voxel-box budget per workgroup, 8..144 KiB;
                                     0 = per view: 144 KiB for views oblique to all three axes, else 64 */
    int32_t slab_max;             /* LDS-staged path: thickest slab tried, 1..64 voxels */
    int32_t copy;                 /* layouts with 3 orientation copies: -1 auto (fastest axis along the
                                     image rows), 0/1/2 force the x/y/z-fastest copy */
    int32_t order;                /* tile order: 0 one contiguous band of tiles per XCD (L2 reuse),
                                     1 hardware order (work spread evenly over the XCDs),
                                     2 4x4-tile blocks per XCD, blocks dealt over the XCDs in turn,
                                     3 (default) LDS-staged path: bundles in decreasing order of their
                                     estimated box fetch, sorted on the device into the workspace
                                     (vr_render_workspace_bytes); without that workspace, and on other
                                     paths, as 1 */
} vr_tuning;

/* ---- context ---------------------------------------------------------- */

/* Create a context bound to HIP device `device`.  device = -1 creates a
 * host-only context: every argument and state check works, and every call
 * that would launch work returns VR_EDEVICE (for hosts without a GPU). */
int vr_create(vr_ctx **out, int device);
int vr_destroy(vr_ctx *ctx);
/* Message of the last failing call on this context (or of the calling
 * thread when ctx is NULL).  Valid until the next call. */
const char *vr_last_error(const vr_ctx *ctx);
const char *vr_version(void);

/* Debug builds (every source compiled with -DVR_DEBUG_BOUNDS; the build
 * writes them as libvrcube_debug.so) check the index range of every direct
 * gather from the volume (padded indices within [0, N + 1]) and of every
 * read of an LDS-staged voxel box, and count violations in a 4-byte device
 * counter the context allocates (the only other allocation of a context).
 * This call waits for the device, returns the count since the previous call
 * and resets it.  Release builds: VR_EUNSUPPORTED.  Host-only context:
 * VR_EDEVICE. */
int64_t vr_debug_bounds_violations(vr_ctx *ctx);

/* ---- volume (section 1: cubes larger than one machine's memory are
 *      handled as bricks; section 3: float32 cubes such as HIPASS) -------- */

/* Bytes of the brick-major storage of an nx*ny*nz cube with brick edge B in
 * `storage` type: ceil(n_a/B) bricks per axis, each holding
 * (min(B,n_a)+2) voxels per axis (a one-voxel apron on every side,
 * clamp-to-edge at the cube's faces), rows padded to a multiple of 8
 * elements: bricks * roundup(Bx+2, 8) * (By+2) * (Bz+2) * element size.
 * B <= 0 means one brick for the whole cube.  orientations = 3 (one-brick
 * layouts only) stores three copies of the padded cube with x, y and z
 * fastest, each 256-byte aligned, so that every view direction finds a copy
 * whose rows run across its ray packets (shear-warp renderers keep such
 * principal-axis copies for the same reason); 1 stores the x-fastest copy
 * only.  An FP32 layout with three copies also stores a line copy for MIP in
 * object order, from the next 128-element boundary: every padded row of the
 * x-fastest copy as ceil((nx+2)/31) lines of 32 elements, line L holding the
 * row's elements 31 L .. 31 L + 31 (the row's last element repeated past its
 * end), (nz+2) * (ny+2) * lines * 32 elements.  Pure host function; returns
 * < 0 on invalid sizes. */
int64_t vr_volume_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t brick_edge,
                        int32_t orientations);

/* Transcode a float32 (nz,ny,nx) C-ordered cube at src_dev into the
 * brick-major layout at dst_dev (dst_bytes >= vr_volume_bytes), converting
 * to FP16/BF16 with round-to-nearest-even when asked.  The context then
 * renders from dst_dev; src_dev may be freed once the stream has passed this
 * call.  Errors: EINVAL (sizes, null pointers, dtype, orientations),
 * ENOMEM (dst too small), EUNSUPPORTED (a brick or copy of 2^32 voxels or
 * more), EDEVICE. */
int vr_load_volume(vr_ctx *ctx, const float *src_dev, int64_t nx, int64_t ny, int64_t nz,
                   int32_t storage, int32_t brick_edge, int32_t orientations, void *dst_dev,
                   int64_t dst_bytes, void *stream);

/* Stream a cube larger than device memory slab by slab: describe the layout
 * once (vr_describe_volume: same arguments as vr_load_volume without the
 * source), then transcode each z-slab [z0, z0+nz_slab) from src_dev, a
 * C-ordered (nz_slab, ny, nx) float32 block holding those planes
 * (vr_load_slab; every plane of the cube must be loaded once before
 * rendering).  vr_load_volume is describe + one slab covering the cube. */
int vr_describe_volume(vr_ctx *ctx, int64_t nx, int64_t ny, int64_t nz, int32_t storage,
                       int32_t brick_edge, int32_t orientations, void *dst_dev, int64_t dst_bytes);
int vr_load_slab(vr_ctx *ctx, const float *src_dev, int64_t z0, int64_t nz_slab, void *stream);

/* ---- out-of-core bricks (section 1: cubes larger than one machine's
 *      memory are rendered brick by brick; section 3: WALLABY's expected
 *      6144 x 6144 x 16384 cube, about nine times one GPU's memory) ------- */

/* Bytes of one brick of the bricked layout (vr_volume_bytes with this brick
 * edge and one orientation, divided by the brick count); < 0 if invalid. */
int64_t vr_brick_bytes(int64_t nx, int64_t ny, int64_t nz, int32_t storage, int32_t brick_edge);

/* Pack a float32 (nz,ny,nx) cube held in host memory into the bricked
 * layout (brick_edge > 0, one orientation) in host memory at dst_host
 * (vr_volume_bytes bytes), with `threads` host threads (0: all cores).  The
 * bytes are those vr_load_volume writes on the device (same apron, padding
 * and round-to-nearest-even).  Pure host; errors through vr_last_error(NULL). */
int vr_pack_bricks_host(const float *src_host, int64_t nx, int64_t ny, int64_t nz, int32_t storage,
                        int32_t brick_edge, void *dst_host, int64_t dst_bytes, int32_t threads);

/* Make the context render a bricked volume whose packed bricks stay in host
 * memory (host_bricks, vr_volume_bytes bytes, borrowed; pinned memory lets
 * the copies run asynchronously) through a device cache of
 * floor(cache_bytes / vr_brick_bytes) brick slots at cache_dev (borrowed).
 * vr_render_bricks then copies every visible brick that is not cached into
 * the least recently used slot on a copy stream of the context's own
 * (overlapping the rendering of the bricks already there), waiting until
 * the slot's previous brick has been rendered; the images are those of the
 * resident volume.  The cache persists across calls until the volume is
 * described again.  Other renders (vr_render, batches, backward) return
 * EUNSUPPORTED on a streamed volume. */
int vr_describe_streamed_volume(vr_ctx *ctx, int64_t nx, int64_t ny, int64_t nz, int32_t storage,
                                int32_t brick_edge, const void *host_bricks, int64_t host_bytes, void *cache_dev,
                                int64_t cache_bytes);

/* Bricks copied from host memory and cache hits so far, and the cache's
 * slot count (any pointer may be NULL). */
int vr_stream_stats(const vr_ctx *ctx, int64_t *bricks_copied, int64_t *cache_hits, int32_t *slots);

/* ---- transfer function (section 2: the colour map) --------------------- */

/* n straight-RGBA float32 entries (n*4 floats on the device, n in [2, 1024])
 * over [vmin, vmax] (vmax > vmin).  Borrowed: must stay valid while used.
 * The call reads the table back once (a blocking copy of n*16 bytes, so the
 * entries must be in place when it is made) to find its largest opacity:
 * that bounds how early a composite ray can stop and picks the kernel of
 * vr_render's automatic path; the images do not depend on it. */
int vr_set_transfer_function(vr_ctx *ctx, const float *rgba_dev, int32_t n, float vmin, float vmax);

/* ---- camera (section 3: a static render keeps the view and takes a new output size) */

int vr_set_camera(vr_ctx *ctx, const vr_camera *cam);

/* ---- render ------------------------------------------------------------ */

/* Workspace bytes vr_render needs for these params with the current camera,
 * volume and launch shape: samples taken and transmittance checkpoints when
 * save_for_backward (int32 per pixel, then from the next 256-byte boundary
 * ceil(max samples / VR_CHECKPOINT_INTERVAL) float planes of one value per
 * pixel); 64 bytes per pixel of ray records when the view is
 * rendered in object order (MIP, path 4 or the automatic choice); when it is
 * rendered by the LDS-staged bundle kernel with tuning order 3, the bundle
 * order: 4 bytes per bundle (from 256-byte boundaries) and 1 byte per bundle;
 * else 0.  With a smaller workspace an object-order view is rendered by the
 * bundle kernels instead, and bundles run in hardware order (the same
 * image either way). */
int64_t vr_render_workspace_bytes(const vr_ctx *ctx, const vr_render_params *params);

/* Render the camera's viewport into out_dev: tile_h*tile_w*4 floats
 * (composite, premultiplied RGBA) or tile_h*tile_w floats (MIP).  Workspace
 * may be NULL when vr_render_workspace_bytes returns 0. */
int vr_render(vr_ctx *ctx, const vr_render_params *params, float *out_dev,
              void *workspace_dev, int64_t ws_bytes, void *stream);

/* vr_render for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation).
 * The only scratch a render needs without save_for_backward, the per-pixel
 * ray records of MIP in object order or the bundle order of the LDS-staged
 * kernel (vr_render_workspace_bytes), lives in a fixed device array of vr_render_noalloc_max_bytes() = 128 MiB (ray records
 * of up to 2^21 pixels), one per GPU, held until the process ends; the call
 * allocates nothing.  The caller still passes the output.  Every call on one
 * GPU shares that GPU's array: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be ordered by the caller.  The
 * records are fully rewritten by each call before they are read.
 * Errors: EINVAL for save_for_backward (checkpoints must outlive the call:
 * use vr_render with a workspace), ENOMEM when the render needs more
 * scratch than the array holds, plus those of vr_render. */
int64_t vr_render_noalloc_max_bytes(void);
int vr_render_noalloc(vr_ctx *ctx, const vr_render_params *params, float *out_dev, void *stream);

/* Samples each pixel's ray takes (up to and including the early stop),
 * int32 per pixel.  Used for throughput denominators; not a hot path. */
int vr_count_samples(vr_ctx *ctx, const vr_render_params *params, int32_t *counts_dev, void *stream);

/* Compulsory-traffic counter: marks every 8x8x8 voxel block touched by the
 * interpolation footprint of a sample actually taken, in a bitmap of
 * ceil(nx/8)*ceil(ny/8)*ceil(nz/8) bits (caller-zeroed, uint32 words) at
 * bitmap_dev.  vr_touched_bitmap_bytes gives its size. */
int64_t vr_touched_bitmap_bytes(const vr_ctx *ctx);
int vr_mark_touched_blocks(vr_ctx *ctx, const vr_render_params *params, uint32_t *bitmap_dev,
                           int64_t bitmap_bytes, void *stream);

/* ---- bricks and sort-last compositing (sections 1 and 3: the volume is
 *      distributed as bricks; partial images are combined) --------------- */

/* Pool bytes vr_render_bricks needs for the current camera and volume:
 * every brick's footprint partial plus a descriptor table. */
int64_t vr_bricks_pool_bytes(const vr_ctx *ctx, const vr_render_params *params);

/* Render every brick of the loaded volume that the viewport sees into its
 * own footprint partial inside pool_dev.  Fills parts[0 .. *n_parts) (host
 * array of capacity max_parts) in brick-id order. */
int vr_render_bricks(vr_ctx *ctx, const vr_render_params *params, vr_partial *parts,
                     int32_t max_parts, int32_t *n_parts, void *pool_dev, int64_t pool_bytes,
                     void *stream);

/* Front-to-back order of partials (host): order_out[i] is the index into
 * parts of the i-th partial to composite. */
int vr_brick_order(const vr_ctx *ctx, const vr_partial *parts, int32_t n, int32_t *order_out);

/* Composite partials in the given order into out_dev (tile_h*tile_w*4, or
 * *1 for MIP where the combination is the maximum).  The workspace holds
 * the descriptor table: vr_composite_workspace_bytes(n). */
int64_t vr_composite_workspace_bytes(int32_t n);
int vr_composite_bricks(vr_ctx *ctx, const vr_render_params *params, const vr_partial *parts,
                        const int32_t *order, int32_t n, float *out_dev, void *workspace_dev,
                        int64_t ws_bytes, void *stream);

/* ---- differentiation ---------------------------------------------------- */

/* Gradients of a scalar loss with respect to the transfer function and the
 * voxels, given dL/d(image) (tile_h*tile_w*4 floats).  Needs the workspace
 * of a vr_render call with save_for_backward = 1 and the same params,
 * camera, volume and table.  Accumulates (+=) into grad_lut_dev (n*4 floats)
 * and grad_vol_dev ((nz,ny,nx) float32, C order); either may be NULL.
 * Composite, trilinear, FP32 storage only. */
int vr_render_backward(vr_ctx *ctx, const vr_render_params *params, const float *grad_out_dev,
                       const void *workspace_dev, int64_t ws_bytes, float *grad_lut_dev,
                       float *grad_vol_dev, void *stream);

/* ---- depth and catalogue overlay (section 2: the box around each source
 *      of a detection catalogue is outlined on top of the rendered image
 *      and moves with the view) ------------------------------------------ */

/* One catalogue entry: the axis-aligned box [lo, hi] in voxel coordinates of
 * the cube (world units; a source covering voxels i0..i1 along an axis spans
 * [i0, i1 + 1]) and its straight RGBA colour (alpha: how strongly it is
 * drawn over the image). */
typedef struct {
    float lo[3], hi[3];
    float rgba[4];
} vr_box;

/* Per-pixel depth of the current view, tile_h*tile_w floats: the ray
 * parameter t (voxels from the ray's origin) of
 *  - composite: the first sample after which the accumulated opacity A
 *    reaches `level` (in (0, 1]), among the samples the render takes (the
 *    early stop included), with the render's own FP32 arithmetic;
 *  - MIP: the first sample whose value equals the ray's maximum;
 * +inf where there is no such sample (a miss, or A never reaches level).
 * One-brick layouts only (EUNSUPPORTED for bricked ones); the params are
 * those of the render the depth belongs to (save_for_backward ignored). */
int vr_render_depth(vr_ctx *ctx, const vr_render_params *params, float level, float *depth_dev, void *stream);

/* Draw n catalogue boxes (boxes_dev: n vr_box on the device) as wireframes
 * over image_dev, the current view's premultiplied RGBA tile (tile_h*tile_w*4
 * floats, modified in place).  A pixel is covered by an edge when its centre
 * lies within half_width pixels (in (0, 64]) of the edge's projection (the
 * part in front of the near plane, 1e-3 voxel before a perspective eye);
 * the edge's depth there is the ray distance of its 3D point under the
 * projected segment's point nearest the centre, and the edge is visible
 * when that depth is at most depth_dev's value at the pixel (depth_dev NULL:
 * every edge is visible; pass vr_render_depth's output to hide edges behind
 * the rendered emission).  Each pixel takes the colour of the nearest
 * visible covering box (ties: the lower index) and becomes
 * rgba.a * (r, g, b, 1) + (1 - a) * pixel. */
int vr_overlay_boxes(vr_ctx *ctx, const vr_box *boxes_dev, int32_t n, float half_width, const float *depth_dev,
                     float *image_dev, void *stream);

/* ---- display pyramid and pyramidal tiled TIFF (section 3: the static
 *      high-resolution render is stored as a TIFF and converted to the
 *      pyramidal tiled TIFF an image server streams to the tiled wall) ---- */

/* Bytes of the display pyramid of a w x h image with square tiles of `tile`
 * pixels (a multiple of 16 in [16, 4096]): level 0 is w x h, level l+1 is
 * ceil(w_l/2) x ceil(h_l/2), and the levels stop at the first one whose
 * sides both fit one tile; every level is RGBA8 (4 bytes per pixel, rows
 * packed), the levels stored one after the other.  *levels_out (may be
 * NULL) gets their number.  Pure host function; < 0 on invalid sizes. */
int64_t vr_pyramid_bytes(int32_t w, int32_t h, int32_t tile, int32_t *levels_out);

/* Build the pyramid of a premultiplied RGBA float image (rgba_dev: h*w*4
 * floats, 16-byte aligned) into dst_dev (vr_pyramid_bytes bytes, 4-byte
 * aligned).  Level 0 per channel: floor(clamp(v, 0, 1) * 255 + 1/2), NaN
 * as 0, computed exactly; level l+1 pixel (x, y): per channel the rounded
 * mean (s + n/2) / n (integer division) of the n <= 4 pixels (2x + a,
 * 2y + b), a, b in {0, 1}, that exist in level l. */
int vr_build_pyramid(vr_ctx *ctx, const float *rgba_dev, int32_t w, int32_t h, int32_t tile, uint8_t *dst_dev,
                     int64_t dst_bytes, void *stream);

/* Write a pyramid (a host copy of vr_build_pyramid's output for the same w,
 * h, tile) to `path` as a pyramidal tiled TIFF: one image file directory per
 * level, chained from full resolution down (NewSubfileType 1 on the reduced
 * levels), tile x tile tiles (zero beyond the image), 8-bit RGBA with
 * associated alpha (the render's premultiplied colour), uncompressed.
 * bigtiff: 0 writes classic TIFF unless the file reaches 4 GiB (then
 * BigTIFF), 1 always BigTIFF.  Host only (no context); errors are reported
 * through vr_last_error(NULL). */
int vr_write_pyramid_tiff(const char *path, const uint8_t *pyramid_host, int32_t w, int32_t h, int32_t tile,
                          int32_t bigtiff);

/* ---- batches (section 3: many viewports / display tiles at once) --------- */

/* Workspace bytes of vr_render_batch for these views (work table + queue). */
int64_t vr_batch_workspace_bytes(const vr_ctx *ctx, const vr_view *views, int32_t n_views);

/* Render n_views views of the loaded volume in one persistent launch.  Each
 * view has its own camera, output and table (luts_dev: n_luts tables of
 * lut_n entries, all over [vmin, vmax]).  use_graph != 0 captures the launch
 * in a HIP graph on first use and replays it while the views' sizes stay the
 * same (cameras and output pointers may change between calls). */
int vr_render_batch(vr_ctx *ctx, const vr_render_params *params, const vr_view *views,
                    int32_t n_views, const float *luts_dev, int32_t n_luts, int32_t lut_n,
                    float vmin, float vmax, void *workspace_dev, int64_t ws_bytes,
                    int32_t use_graph, void *stream);

/* Graphs captured so far by vr_render_batch on this context (a replay with
 * unchanged launch arguments does not capture again). */
int vr_batch_graph_captures(const vr_ctx *ctx);

/* ---- tuning ------------------------------------------------------------- */

/* Current launch shape, and an explicit override (validated). */
int vr_get_tuning(const vr_ctx *ctx, vr_tuning *out);
int vr_set_tuning(vr_ctx *ctx, const vr_tuning *t);

/* Time the candidate launch shapes on the current volume, camera and table
 * (rendering into out_dev with workspace ws), keep the fastest, and record it
 * in the JSON cache at cache_path (keyed by arch, storage type, cube shape
 * and output-size bucket) when cache_path is not NULL.  A cache hit skips
 * the search.  Synchronises the stream. */
int vr_autotune(vr_ctx *ctx, const vr_render_params *params, float *out_dev, void *workspace_dev,
                int64_t ws_bytes, const char *cache_path, void *stream);

/* The same search for vr_render_batch over these views (bundle shape, LDS
 * budget, slab thickness and persistent workgroups per CU), keyed by the
 * batch's total pixel count bucket.  Renders into the views' outputs. */
int vr_autotune_batch(vr_ctx *ctx, const vr_render_params *params, const vr_view *views, int32_t n_views,
                      const float *luts_dev, int32_t n_luts, int32_t lut_n, float vmin, float vmax,
                      void *workspace_dev, int64_t ws_bytes, const char *cache_path, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
