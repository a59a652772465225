// k_march.hip -- K1/K2: single-pass ray march of one viewport.
//
// One lane owns one pixel's ray; a 64-lane wave owns a packet of
// packet_w x packet_h neighbouring pixels, so its rays stay close together
// and their gathers hit the same cache lines.  Ray set-up (camera, clip,
// sample count, first sample position) is FP64, once per ray; the march
// itself advances a signed 32.32 fixed-point position by an exact integer
// increment per sample (no drift from repeated FP32 additions, and the
// integer part is the voxel index), and does all sampling, table and
// compositing arithmetic in FP32.  Samples read the brick-major layout; the
// one-voxel apron makes the 8 trilinear corners of any sample inside a brick
// sit at fixed offsets, and reproduces clamp-to-edge at the cube's faces.
#include "vr_internal.h"

namespace vr {

template <typename S, int FILTER, bool SINGLE>
struct Walker {
    const S *base;        // element 0 of the current brick
    int32_t org[3];       // global index of the brick's local (0,0,0)
    int32_t lim[3];       // local index must stay in [0, lim]
    uint32_t sx, sy, sz;  // element strides of x, y, z

    __device__ __forceinline__ void enter(const VolDev &v, int32_t gx, int32_t gy, int32_t gz) {
        sx = (uint32_t)v.sx;
        sy = (uint32_t)v.sy;
        sz = (uint32_t)v.sz;
        if (SINGLE) {
            base = (const S *)v.data;
            org[0] = org[1] = org[2] = -1;
            lim[0] = v.Bx; lim[1] = v.By; lim[2] = v.Bz;
            return;
        }
        int32_t b[3];
        int32_t g[3] = {gx, gy, gz}, B[3] = {v.Bx, v.By, v.Bz}, nb[3] = {v.nbx, v.nby, v.nbz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int32_t c = (g[a] + 1) / B[a];
            c = g[a] + 1 < 0 ? 0 : c;
            b[a] = min(max(c, 0), nb[a] - 1);
            org[a] = b[a] * B[a] - 1;
        }
        lim[0] = v.Bx; lim[1] = v.By; lim[2] = v.Bz;
        base = (const S *)v.data + ((int64_t)(b[2] * v.nby + b[1]) * v.nbx + b[0]) * v.brick_elems;
    }

    // Value at corner-grid index (ix, iy, iz) (global) with fractions f.
    __device__ __forceinline__ float sample(const VolDev &v, int32_t gx, int32_t gy, int32_t gz,
                                            float fx, float fy, float fz) {
        int32_t lx = gx - org[0], ly = gy - org[1], lz = gz - org[2];
        if (!SINGLE) {
            if ((uint32_t)lx > (uint32_t)lim[0] || (uint32_t)ly > (uint32_t)lim[1] ||
                (uint32_t)lz > (uint32_t)lim[2]) {
                enter(v, gx, gy, gz);
                lx = gx - org[0]; ly = gy - org[1]; lz = gz - org[2];
            }
        }
        const S *p = base + ((uint32_t)lz * sz + (uint32_t)ly * sy + (uint32_t)lx * sx);
        if (FILTER == VR_NEAREST) return Store<S>::ld(p);
        float c000 = Store<S>::ld(p), c100 = Store<S>::ld(p + sx);
        float c010 = Store<S>::ld(p + sy), c110 = Store<S>::ld(p + sy + sx);
        const S *q = p + sz;
        float c001 = Store<S>::ld(q), c101 = Store<S>::ld(q + sx);
        float c011 = Store<S>::ld(q + sy), c111 = Store<S>::ld(q + sy + sx);
        float x00 = fmaf(fx, c100 - c000, c000), x10 = fmaf(fx, c110 - c010, c010);
        float x01 = fmaf(fx, c101 - c001, c001), x11 = fmaf(fx, c111 - c011, c011);
        float y0 = fmaf(fy, x10 - x00, x00), y1 = fmaf(fy, x11 - x01, x01);
        return fmaf(fz, y1 - y0, y0);
    }
};

// Pixel of this lane for the packet layout; false if outside the tile.
__device__ __forceinline__ bool lane_pixel(const MarchArgs &A, int &px, int &py) {
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t gx, gy;
    tile_xy(blockIdx.x, gridDim.x, A.groups_x, (int32_t)(gridDim.x / (uint32_t)A.groups_x), A.order, A.tile_perm,
            gx, gy);
    px = gx * A.packet_w + lane % A.packet_w;
    py = (gy * A.waves + wave) * A.packet_h + lane / A.packet_w;
    return px < A.cam.tile_w && py < A.cam.tile_h;
}

template <typename S, int MODE, int FILTER, bool SINGLE>
__global__ __launch_bounds__(512) void k_march(MarchArgs A) {
    __shared__ float4 lut[1024];
    int px, py;
    const bool valid = lane_pixel(A, px, py);
    int64_t pix = (int64_t)py * A.cam.tile_w + px;

    Ray r{};
    if (valid) make_ray(A.cam, A.vol, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    const int32_t n = r.n;
    int64_t Q[3], D[3];
    fix_start(r, A.step, 0, FILTER == VR_TRILINEAR ? 0.5 : 0.0, Q, D);
    // the table goes to LDS after the FP64 set-up, whose inputs then need not
    // stay live across the copy loop
    if (MODE == VR_COMPOSITE) {
        for (int i = threadIdx.x; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
        __syncthreads();
    }
    if (!valid) return;

    Walker<S, FILTER, SINGLE> w;
    w.enter(A.vol, fix_int(Q[0]), fix_int(Q[1]), fix_int(Q[2]));

    float m = -INFINITY;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    // log-space transmittance: L = sum log1p(-a), compensated
    const bool use_log = (MODE == VR_COMPOSITE) && (A.trans == 1 || (A.trans == 2 && n > 1024));
    LogTrans lt;
    int32_t k = 0;
    for (; k < n; ++k) {
        float fx = 0.f, fy = 0.f, fz = 0.f;
        if (FILTER == VR_TRILINEAR) { fx = fix_frac(Q[0]); fy = fix_frac(Q[1]); fz = fix_frac(Q[2]); }
        float s = w.sample(A.vol, fix_int(Q[0]), fix_int(Q[1]), fix_int(Q[2]), fx, fy, fz);
        Q[0] += D[0]; Q[1] += D[1]; Q[2] += D[2];
        if (MODE == VR_MIP) {
            m = fmaxf(m, s);
        } else {
            if (A.ckpt && (k & (kCkpt - 1)) == 0 && (k >> kCkptShift) < A.ckpt_segs) A.ckpt[(int64_t)(k >> kCkptShift) * A.cam.tile_w * A.cam.tile_h + pix] = T;
            float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
            float ta = T * c.w;
            C0 = fmaf(ta, c.x, C0);
            C1 = fmaf(ta, c.y, C1);
            C2 = fmaf(ta, c.z, C2);
            T = use_log ? lt.step(c.w) : T - ta;
            if (A.ert && T <= A.thr) { ++k; break; }
        }
    }
    if (A.out) {
        if (MODE == VR_MIP) ((float *)A.out)[pix] = m;
        else ((float4 *)A.out)[pix] = make_float4(C0, C1, C2, 1.0f - T);
    }
    if (A.counts) A.counts[pix] = k;
    if (A.taken) A.taken[pix] = k;
}

// Direct march of one lane's ray over a one-brick layout, U samples per
// loop iteration: the 8U gathers of a block are issued together, so a wave
// keeps U times more loads in flight (this path is bound by load latency,
// not arithmetic).  The ray is set up; the table (composite) is in LDS.
template <typename S, int MODE, int FILTER, int U>
__device__ __forceinline__ void march_u_run(const MarchArgs &A, const float4 *lut, const Ray &r, int64_t pix,
                                            int64_t npix) {
    const int32_t n = r.n;
    int64_t Q[3], D[3];
    fix_start(r, A.step, 0, FILTER == VR_TRILINEAR ? 0.5 : 0.0, Q, D);
    float m = -INFINITY;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    const bool use_log = (MODE == VR_COMPOSITE) && (A.trans == 1 || (A.trans == 2 && n > 1024));
    LogTrans lt;
    int32_t k = 0;
    bool stop = false;
    while (k < n && !stop) {
        const int32_t cnt = min(U, n - k);
        float v[U];
        int64_t q0 = Q[0], q1 = Q[1], q2 = Q[2];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
            if (FILTER == VR_TRILINEAR) { fx = fix_frac(q0); fy = fix_frac(q1); fz = fix_frac(q2); }
            v[j] = j < cnt ? gsample<S, FILTER>(A.vol, fix_int(q0), fix_int(q1), fix_int(q2), fx, fy, fz) : 0.0f;
            q0 += D[0]; q1 += D[1]; q2 += D[2];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (j >= cnt || stop) break;
            const float s = v[j];
            if (MODE == VR_MIP) {
                m = fmaxf(m, s);
            } else {
                if (A.ckpt && ((k + j) & (kCkpt - 1)) == 0 && ((k + j) >> kCkptShift) < A.ckpt_segs)
                    A.ckpt[(int64_t)((k + j) >> kCkptShift) * npix + pix] = T;
                float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
                float ta = T * c.w;
                C0 = fmaf(ta, c.x, C0);
                C1 = fmaf(ta, c.y, C1);
                C2 = fmaf(ta, c.z, C2);
                T = use_log ? lt.step(c.w) : T - ta;
                if (A.ert && T <= A.thr) { stop = true; k += j + 1; }
            }
        }
        if (!stop) {
            k += cnt;
            Q[0] = q0; Q[1] = q1; Q[2] = q2;
        }
    }
    if (A.out) {
        if (MODE == VR_MIP) ((float *)A.out)[pix] = m;
        else ((float4 *)A.out)[pix] = make_float4(C0, C1, C2, 1.0f - T);
    }
    if (A.counts) A.counts[pix] = k;
    if (A.taken) A.taken[pix] = k;
}

template <typename S, int MODE, int FILTER, int U>
__global__ __launch_bounds__(256) void k_march_u(MarchArgs A) {
    __shared__ float4 lut[1024];
    int px, py;
    const bool valid = lane_pixel(A, px, py);
    const int64_t pix = (int64_t)py * A.cam.tile_w + px;
    const int64_t npix = (int64_t)A.cam.tile_w * A.cam.tile_h;
    Ray r{};
    if (valid) make_ray(A.cam, A.vol, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    // the table goes to LDS after the FP64 set-up
    if (MODE == VR_COMPOSITE) {
        for (int i = threadIdx.x; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
        __syncthreads();
    }
    if (!valid) return;
    march_u_run<S, MODE, FILTER, U>(A, lut, r, pix, npix);
}

// K1/K2, compacting form (one-brick layouts).  A workgroup owns a share of
// `share` consecutive packets (row-major over the tile) and its waves keep 64
// rays in flight each.  A pass takes up to U samples of every live ray (the
// gathers of a pass issued together); a lane whose ray has ended writes its
// pixel and goes idle.  When a ballot shows at most refill_at live lanes, the
// idle lanes take the next pixels of the share from a counter in LDS, each
// ranked by a count of the idle lanes below it, so rays that stop early (the
// opacity threshold, short chords near the cube's edges, misses) do not hold
// lanes idle while the longest ray of a fixed packet finishes.  Pixel i of
// the share is lane i%64 of its packet i/64.  Same per-ray arithmetic as
// march_u_run, so the images are identical.  A wave leaves the loop once the
// counter has passed the share's last pixel and its lanes are idle; every
// pass of the loop takes a sample or advances the counter.
template <typename S, int MODE, int FILTER, int U>
__global__ __launch_bounds__(256) void k_march_c(CompactArgs C) {
    __shared__ float4 lut[1024];
    __shared__ uint32_t next;     // the share's pixel counter
    const MarchArgs &A = C.m;
    if (threadIdx.x == 0) next = 0u;
    if (MODE == VR_COMPOSITE)
        for (int i = threadIdx.x; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t npix = (int64_t)A.cam.tile_w * A.cam.tile_h;
    const int32_t p_first = (int32_t)blockIdx.x * C.share;
    const int32_t n_share = min(C.share, C.packets - p_first) * 64;   // pixels of this share
    const double h = FILTER == VR_TRILINEAR ? 0.5 : 0.0;
    int64_t Q[3] = {0, 0, 0}, D[3] = {0, 0, 0};
    int32_t n = 0, k = 0;
    int64_t pix = 0;
    float m = -INFINITY, T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    LogTrans lt;
    bool use_log = false, live = false;
    bool drained = false;         // the counter has passed the share's last pixel (uniform)
    auto finish = [&]() {
        if (A.out) {
            if (MODE == VR_MIP) ((float *)A.out)[pix] = m;
            else ((float4 *)A.out)[pix] = make_float4(C0, C1, C2, 1.0f - T);
        }
        if (A.counts) A.counts[pix] = k;
        if (A.taken) A.taken[pix] = k;
    };
    for (;;) {
        uint64_t lv = __ballot(live);
        if (__popcll(lv) <= C.refill_at && !drained) {
            const uint64_t idle = ~lv;
            const int32_t nidle = __popcll(idle);
            const int32_t rank = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
            uint32_t got = 0;
            if (lane == 0) got = atomicAdd(&next, (uint32_t)nidle);
            got = (uint32_t)__shfl((int)got, 0, 64);
            if ((int64_t)got + nidle >= n_share) drained = true;
            const int32_t i = (int32_t)got + rank;
            if (!live && i < n_share) {
                const int32_t p = p_first + (i >> 6), j = i & 63;
                const int px = (p % C.gxn) * A.packet_w + j % A.packet_w;
                const int py = (p / C.gxn) * A.packet_h + j / A.packet_w;
                if (px < A.cam.tile_w && py < A.cam.tile_h) {
                    Ray r{};
                    make_ray(A.cam, A.vol, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
                    fix_start(r, A.step, 0, h, Q, D);
                    n = r.n;
                    k = 0;
                    pix = (int64_t)py * A.cam.tile_w + px;
                    m = -INFINITY;
                    T = 1.0f;
                    C0 = C1 = C2 = 0.0f;
                    lt = LogTrans();
                    use_log = (MODE == VR_COMPOSITE) && (A.trans == 1 || (A.trans == 2 && n > 1024));
                    if (n > 0) live = true;
                    else finish();
                }
            }
            lv = __ballot(live);
        }
        if (lv == 0) {
            if (drained) break;
            continue;
        }
        if (!live) continue;
        const int32_t cnt = min(U, n - k);
        float v[U];
        int64_t q0 = Q[0], q1 = Q[1], q2 = Q[2];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
            if (FILTER == VR_TRILINEAR) { fx = fix_frac(q0); fy = fix_frac(q1); fz = fix_frac(q2); }
            v[j] = j < cnt ? gsample<S, FILTER>(A.vol, fix_int(q0), fix_int(q1), fix_int(q2), fx, fy, fz) : 0.0f;
            q0 += D[0]; q1 += D[1]; q2 += D[2];
        }
        bool stop = false;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (j >= cnt || stop) break;
            const float s = v[j];
            if (MODE == VR_MIP) {
                m = fmaxf(m, s);
            } else {
                if (A.ckpt && ((k + j) & (kCkpt - 1)) == 0 && ((k + j) >> kCkptShift) < A.ckpt_segs)
                    A.ckpt[(int64_t)((k + j) >> kCkptShift) * npix + pix] = T;
                float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
                float ta = T * c.w;
                C0 = fmaf(ta, c.x, C0);
                C1 = fmaf(ta, c.y, C1);
                C2 = fmaf(ta, c.z, C2);
                T = use_log ? lt.step(c.w) : T - ta;
                if (A.ert && T <= A.thr) { stop = true; k += j + 1; }
            }
        }
        if (!stop) {
            k += cnt;
            Q[0] = q0; Q[1] = q1; Q[2] = q2;
        }
        if (stop || k >= n) {
            finish();
            live = false;
        }
    }
}

// K6, direct form: persistent workgroups pull (view, tile) items from the
// same atomic queue as the LDS-staged batch kernel (views largest first) and
// march each tile's rays with direct gathers; the table of the item's view is
// reloaded into LDS when it changes.  Serves batches of early-stopping
// composites, whose rays take few samples.  Each workgroup exits once the
// counter passes the item count.
template <typename S, int MODE, int FILTER, int U>
__global__ __launch_bounds__(512) void k_batch_direct(BatchArgs B) {
    __shared__ float4 lut[1024];
    __shared__ int32_t item_s;
    int32_t cur_lut = -1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ph = 64 / B.bw;                     // packet rows: bw x ph pixels per wave
    for (;;) {
        if (threadIdx.x == 0) item_s = (int32_t)atomicAdd(B.queue, 1u);
        __syncthreads();
        const int32_t item = item_s;
        if (item >= B.total_items) break;
        int32_t lo = 0, hi = B.n_views - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (B.views[mid].tile_begin <= item) lo = mid;
            else hi = mid - 1;
        }
        const ViewDev &V = B.views[lo];
        if (MODE == VR_COMPOSITE && V.lut_index != cur_lut) {
            const float4 *src = B.luts + (int64_t)V.lut_index * B.lut_n;
            for (int i = threadIdx.x; i < B.lut_n; i += blockDim.x) lut[i] = src[i];
            cur_lut = V.lut_index;
        }
        __syncthreads();   // table in place; item_s is rewritten only after the next barrier
        MarchArgs A{};
        A.cam = V.cam;
        A.vol = B.vol;
        A.vol.data = V.vdata;
        A.vol.sx = V.vsx;
        A.vol.sy = V.vsy;
        A.vol.sz = V.vsz;
        A.vol.ori = V.ori;
        A.lut.n = B.lut_n;
        A.lut.vmin = B.vmin;
        A.lut.scale = B.scale;
        A.step = B.step;
        A.thr = B.thr;
        A.ert = B.ert;
        A.trans = B.trans;
        A.out = V.out;
        const int32_t t = item - V.tile_begin;
        const int px = (t % V.tiles_x) * B.bw + lane % B.bw;
        const int py = (t / V.tiles_x) * B.bh + wave * ph + lane / B.bw;
        if (px < A.cam.tile_w && py < A.cam.tile_h) {
            Ray r{};
            make_ray(A.cam, A.vol, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
            march_u_run<S, MODE, FILTER, U>(A, lut, r, (int64_t)py * A.cam.tile_w + px,
                                            (int64_t)A.cam.tile_w * A.cam.tile_h);
        }
    }
}

template <typename S, int MODE, int FILTER>
static hipError_t launch_batch_direct_u(const BatchArgs &a, int32_t unroll, int32_t groups, hipStream_t s) {
    const dim3 g((unsigned)groups), b((unsigned)(a.bw * a.bh));
    if (unroll == 4) hipLaunchKernelGGL((k_batch_direct<S, MODE, FILTER, 4>), g, b, 0, s, a);
    else if (unroll == 2) hipLaunchKernelGGL((k_batch_direct<S, MODE, FILTER, 2>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_batch_direct<S, MODE, FILTER, 1>), g, b, 0, s, a);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_batch_direct_s(const BatchArgs &a, int32_t mode, int32_t filter, int32_t unroll,
                                        int32_t groups, hipStream_t s) {
    if (mode == VR_MIP) {
        if (filter == VR_NEAREST) return launch_batch_direct_u<S, VR_MIP, VR_NEAREST>(a, unroll, groups, s);
        return launch_batch_direct_u<S, VR_MIP, VR_TRILINEAR>(a, unroll, groups, s);
    }
    if (filter == VR_NEAREST) return launch_batch_direct_u<S, VR_COMPOSITE, VR_NEAREST>(a, unroll, groups, s);
    return launch_batch_direct_u<S, VR_COMPOSITE, VR_TRILINEAR>(a, unroll, groups, s);
}

hipError_t launch_batch_direct(const BatchArgs &a, int32_t mode, int32_t filter, int32_t unroll, int32_t groups,
                               hipStream_t s) {
    if (groups <= 0 || a.total_items <= 0) return hipSuccess;
    if (a.bw * a.bh > 512 || 64 % a.bw != 0 || a.bh % (64 / a.bw) != 0) return hipErrorInvalidValue;
    switch (a.vol.dtype) {
        case VR_F32: return launch_batch_direct_s<float>(a, mode, filter, unroll, groups, s);
        case VR_F16: return launch_batch_direct_s<_Float16>(a, mode, filter, unroll, groups, s);
        default: return launch_batch_direct_s<bf16_t>(a, mode, filter, unroll, groups, s);
    }
}

// K7: mark the 8^3 blocks touched by each taken sample's interpolation
// footprint (measurement only, not timed).  Same traversal and stop rule as
// k_march.
template <typename S>
__global__ __launch_bounds__(256) void k_touch(MarchArgs A, int32_t mode, int32_t filter, uint32_t *bits) {
    __shared__ float4 lut[1024];
    for (int i = threadIdx.x; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
    __syncthreads();
    int px, py;
    if (!lane_pixel(A, px, py)) return;
    Ray r;
    make_ray(A.cam, A.vol, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    int64_t Q[3], D[3];
    fix_start(r, A.step, 0, filter == VR_TRILINEAR ? 0.5 : 0.0, Q, D);
    const int nbx = (A.vol.nx + 7) / 8, nby = (A.vol.ny + 7) / 8;
    const int32_t N[3] = {A.vol.nx, A.vol.ny, A.vol.nz};
    Walker<S, VR_TRILINEAR, false> wt;
    Walker<S, VR_NEAREST, false> wn;
    wt.enter(A.vol, fix_int(Q[0]), fix_int(Q[1]), fix_int(Q[2]));
    wn.enter(A.vol, fix_int(Q[0]), fix_int(Q[1]), fix_int(Q[2]));
    int b0l[3] = {-1, -1, -1}, b1l[3] = {-1, -1, -1};
    float T = 1.0f;
    for (int32_t k = 0; k < r.n; ++k) {
        int32_t i[3], b0[3], b1[3];
        bool same = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            i[a] = fix_int(Q[a]);
            int lo = min(max(i[a], 0), N[a] - 1);
            int hi = filter == VR_TRILINEAR ? min(max(i[a] + 1, 0), N[a] - 1) : lo;
            b0[a] = lo >> 3;
            b1[a] = hi >> 3;
            same = same && b0[a] == b0l[a] && b1[a] == b1l[a];
        }
        if (!same) {
            for (int z = b0[2]; z <= b1[2]; ++z)
                for (int y = b0[1]; y <= b1[1]; ++y)
                    for (int x = b0[0]; x <= b1[0]; ++x) {
                        int64_t id = ((int64_t)z * nby + y) * nbx + x;
                        atomicOr(bits + (id >> 5), 1u << (id & 31));
                    }
#pragma unroll
            for (int a = 0; a < 3; ++a) { b0l[a] = b0[a]; b1l[a] = b1[a]; }
        }
        if (mode == VR_COMPOSITE && A.ert) {
            float s;
            if (filter == VR_TRILINEAR)
                s = wt.sample(A.vol, i[0], i[1], i[2], fix_frac(Q[0]), fix_frac(Q[1]), fix_frac(Q[2]));
            else
                s = wn.sample(A.vol, i[0], i[1], i[2], 0.f, 0.f, 0.f);
            float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
            T = T - T * c.w;
            if (T <= A.thr) break;
        }
        Q[0] += D[0]; Q[1] += D[1]; Q[2] += D[2];
    }
}

template <typename S, int MODE, int FILTER>
static void launch_one(const MarchArgs &a, dim3 g, dim3 b, hipStream_t s) {
    if (a.vol.single && b.x <= 256 && a.unroll == 2)
        hipLaunchKernelGGL((k_march_u<S, MODE, FILTER, 2>), g, b, 0, s, a);
    else if (a.vol.single && b.x <= 256 && a.unroll == 4)
        hipLaunchKernelGGL((k_march_u<S, MODE, FILTER, 4>), g, b, 0, s, a);
    else if (a.vol.single) hipLaunchKernelGGL((k_march<S, MODE, FILTER, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_march<S, MODE, FILTER, false>), g, b, 0, s, a);
}

template <typename S>
static void launch_s(const MarchArgs &a, int32_t mode, int32_t filter, dim3 g, dim3 b, hipStream_t s) {
    if (mode == VR_MIP) {
        if (filter == VR_NEAREST) launch_one<S, VR_MIP, VR_NEAREST>(a, g, b, s);
        else launch_one<S, VR_MIP, VR_TRILINEAR>(a, g, b, s);
    } else {
        if (filter == VR_NEAREST) launch_one<S, VR_COMPOSITE, VR_NEAREST>(a, g, b, s);
        else launch_one<S, VR_COMPOSITE, VR_TRILINEAR>(a, g, b, s);
    }
}

static void grid_of(const MarchArgs &a, dim3 &g, dim3 &b) {
    int gy = (a.cam.tile_h + a.packet_h * a.waves - 1) / (a.packet_h * a.waves);
    g = dim3((unsigned)(a.groups_x * gy));
    b = dim3((unsigned)(64 * a.waves));
}

hipError_t launch_march(const MarchArgs &a, int32_t mode, int32_t filter, hipStream_t s) {
    dim3 g, b;
    grid_of(a, g, b);
    if (g.x == 0) return hipSuccess;
    switch (a.vol.dtype) {
        case VR_F32: launch_s<float>(a, mode, filter, g, b, s); break;
        case VR_F16: launch_s<_Float16>(a, mode, filter, g, b, s); break;
        default: launch_s<bf16_t>(a, mode, filter, g, b, s); break;
    }
    return hipGetLastError();
}

template <typename S, int MODE, int FILTER>
static void launch_compact_u(const CompactArgs &c, dim3 g, dim3 b, hipStream_t s) {
    if (c.m.unroll == 4) hipLaunchKernelGGL((k_march_c<S, MODE, FILTER, 4>), g, b, 0, s, c);
    else if (c.m.unroll == 2) hipLaunchKernelGGL((k_march_c<S, MODE, FILTER, 2>), g, b, 0, s, c);
    else hipLaunchKernelGGL((k_march_c<S, MODE, FILTER, 1>), g, b, 0, s, c);
}

template <typename S>
static void launch_compact_s(const CompactArgs &c, int32_t mode, int32_t filter, dim3 g, dim3 b, hipStream_t s) {
    if (mode == VR_MIP) {
        if (filter == VR_NEAREST) launch_compact_u<S, VR_MIP, VR_NEAREST>(c, g, b, s);
        else launch_compact_u<S, VR_MIP, VR_TRILINEAR>(c, g, b, s);
    } else {
        if (filter == VR_NEAREST) launch_compact_u<S, VR_COMPOSITE, VR_NEAREST>(c, g, b, s);
        else launch_compact_u<S, VR_COMPOSITE, VR_TRILINEAR>(c, g, b, s);
    }
}

hipError_t launch_march_compact(const MarchArgs &a, int32_t mode, int32_t filter, int32_t packets_per_wave,
                                hipStream_t s) {
    if (!a.vol.single || a.waves < 1 || a.waves > 4 || packets_per_wave < 1 || packets_per_wave > 32 ||
        a.packet_w * a.packet_h != 64)
        return hipErrorInvalidValue;
    CompactArgs c{};
    c.m = a;
    c.gxn = (a.cam.tile_w + a.packet_w - 1) / a.packet_w;
    const int64_t gyn = (a.cam.tile_h + a.packet_h - 1) / a.packet_h;
    const int64_t packets = (int64_t)c.gxn * gyn;
    if (packets * 64 > 0x7fffffffLL) return hipErrorInvalidValue;
    c.packets = (int32_t)packets;
    c.share = a.waves * packets_per_wave;
    c.refill_at = kCompactRefillAt;
    if (packets == 0) return hipSuccess;
    const dim3 g((unsigned)((packets + c.share - 1) / c.share)), b((unsigned)(64 * a.waves));
    switch (a.vol.dtype) {
        case VR_F32: launch_compact_s<float>(c, mode, filter, g, b, s); break;
        case VR_F16: launch_compact_s<_Float16>(c, mode, filter, g, b, s); break;
        default: launch_compact_s<bf16_t>(c, mode, filter, g, b, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_touch(const MarchArgs &a, int32_t mode, int32_t filter, uint32_t *bitmap, hipStream_t s) {
    MarchArgs t = a;
    t.waves = 4;
    t.packet_w = 8;
    t.packet_h = 8;
    t.groups_x = (t.cam.tile_w + 7) / 8;
    dim3 g, b;
    grid_of(t, g, b);
    if (g.x == 0) return hipSuccess;
    switch (t.vol.dtype) {
        case VR_F32: hipLaunchKernelGGL(k_touch<float>, g, b, 0, s, t, mode, filter, bitmap); break;
        case VR_F16: hipLaunchKernelGGL(k_touch<_Float16>, g, b, 0, s, t, mode, filter, bitmap); break;
        default: hipLaunchKernelGGL(k_touch<bf16_t>, g, b, 0, s, t, mode, filter, bitmap); break;
    }
    return hipGetLastError();
}

}  // namespace vr
