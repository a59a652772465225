// k_bricks.hip -- K3 (per-brick partial images) and K4 (sort-last "over"
// composite of the partials).
//
// K3: one 256-thread workgroup per 16x16 pixel tile of one brick's screen
// footprint.  Each lane clips its ray to the brick and takes exactly the
// samples of the global sample grid whose position lies in the brick
// (exact integer membership on the 32.32 fixed-point positions, half-open
// boxes, the cube's far faces belonging to the last brick), marching them
// with direct gathers from that brick's apron-padded block.  Early
// termination is per brick.  The partial holds premultiplied RGBA (or the
// brick's maximum in MIP mode).
//
// K4: one workgroup per 16x16 output tile walks the partial rectangles in
// visibility order (uniform rectangle tests) and composites the covered
// pixels front to back, C += (1 - A) C_b, A += (1 - A) A_b (maximum in MIP).
#include "vr_internal.h"

namespace vr {

template <typename S, int MODE, int FILTER>
__global__ __launch_bounds__(256) void k_brick(MarchArgs A, const BrickJob *__restrict__ jobs, int32_t n_jobs) {
    __shared__ float4 lut[1024];
    // job of this tile (binary search on tile_begin)
    const int32_t t = blockIdx.x;
    int32_t lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const BrickJob J = jobs[lo];
    const int32_t tl = t - J.tile_begin;
    const int32_t lx = (tl % J.tiles_x) * 16 + (threadIdx.x & 15), ly = (tl / J.tiles_x) * 16 + (threadIdx.x >> 4);
    const bool valid = lx < J.w && ly < J.h;
    const int px = J.x0 + lx, py = J.y0 + ly;
    const VolDev &V = A.vol;

    Ray r{};
    if (valid) make_ray(A.cam, V, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    int64_t P[3], D[3];
    fix_start(r, A.step, 0, 0.0, P, D);
    // this brick's samples: positions in [lo, hi) per axis (far cube faces closed)
    int64_t k0 = 0, k1 = r.n;
    {
        const int64_t one = (int64_t)1 << 32;
        const int32_t bl[3] = {J.bx * V.Bx, J.by * V.By, J.bz * V.Bz};
        const int32_t bh[3] = {min(bl[0] + V.Bx, V.nx), min(bl[1] + V.By, V.ny), min(bl[2] + V.Bz, V.nz)};
        const int32_t N[3] = {V.nx, V.ny, V.nz};
        if (k1 > 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                int64_t a0 = k0, a1 = k1;
                // the cube's outer faces are open-ended (rounding never drops a sample)
                const int64_t lo_f = bl[a] == 0 ? INT64_MIN / 4 : (int64_t)bl[a] * one;
                const int64_t hi_f = bh[a] == N[a] ? INT64_MAX / 4 : (int64_t)bh[a] * one;
                brick_axis_range(P[a], D[a], lo_f, hi_f, a0, a1);
                k0 = max(k0, a0);
                k1 = min(k1, a1);
            }
        }
    }
    if (MODE == VR_COMPOSITE) {
        for (int i = threadIdx.x; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
        __syncthreads();
    }
    if (!valid) return;

    const int64_t sh = FILTER == VR_TRILINEAR ? ((int64_t)1 << 31) : 0;   // corner grid q = p - 1/2
    int64_t Q[3] = {P[0] - sh + k0 * D[0], P[1] - sh + k0 * D[1], P[2] - sh + k0 * D[2]};
    const S *base = J.brick ? (const S *)J.brick
                            : (const S *)V.data + ((int64_t)(J.bz * V.nby + J.by) * V.nbx + J.bx) * V.brick_elems;
    const int32_t ox = J.bx * V.Bx - 1, oy = J.by * V.By - 1, oz = J.bz * V.Bz - 1;
    const uint32_t Px = (uint32_t)V.Px, PxPy = (uint32_t)V.Px * (uint32_t)V.Py;
    const uint32_t lim_x = V.Bx + 1, lim_y = V.By + 1, lim_z = V.Bz + 1;

    float m = -INFINITY;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    for (int64_t k = k0; k < k1; ++k) {
        // local (apron-padded) indices; the clamp keeps reads inside the brick
        uint32_t ix = min((uint32_t)max(fix_int(Q[0]) - ox, 0), lim_x - (FILTER == VR_TRILINEAR));
        uint32_t iy = min((uint32_t)max(fix_int(Q[1]) - oy, 0), lim_y - (FILTER == VR_TRILINEAR));
        uint32_t iz = min((uint32_t)max(fix_int(Q[2]) - oz, 0), lim_z - (FILTER == VR_TRILINEAR));
        const S *p = base + (iz * PxPy + iy * Px + ix);
        float s;
        if (FILTER == VR_NEAREST) {
            s = Store<S>::ld(p);
        } else {
            float fx = fix_frac(Q[0]), fy = fix_frac(Q[1]), fz = fix_frac(Q[2]);
            float c000 = Store<S>::ld(p), c100 = Store<S>::ld(p + 1);
            float c010 = Store<S>::ld(p + Px), c110 = Store<S>::ld(p + Px + 1);
            const S *q = p + PxPy;
            float c001 = Store<S>::ld(q), c101 = Store<S>::ld(q + 1);
            float c011 = Store<S>::ld(q + Px), c111 = Store<S>::ld(q + Px + 1);
            float x00 = fmaf(fx, c100 - c000, c000), x10 = fmaf(fx, c110 - c010, c010);
            float x01 = fmaf(fx, c101 - c001, c001), x11 = fmaf(fx, c111 - c011, c011);
            float y0 = fmaf(fy, x10 - x00, x00), y1 = fmaf(fy, x11 - x01, x01);
            s = fmaf(fz, y1 - y0, y0);
        }
        Q[0] += D[0]; Q[1] += D[1]; Q[2] += D[2];
        if (MODE == VR_MIP) {
            m = fmaxf(m, s);
        } else {
            float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
            float ta = T * c.w;
            C0 = fmaf(ta, c.x, C0);
            C1 = fmaf(ta, c.y, C1);
            C2 = fmaf(ta, c.z, C2);
            T = T - ta;
            if (A.ert && T <= A.thr) break;
        }
    }
    const int64_t o = (int64_t)ly * J.w + lx;
    if (MODE == VR_MIP) J.data[o] = m;
    else ((float4 *)J.data)[o] = make_float4(C0, C1, C2, 1.0f - T);
}

// K4: front-to-back "over" of the partial rectangles (already in visibility
// order) for one 16x16 output tile.  The rectangles are read 256 at a time;
// the ones that touch the tile are compacted into LDS in their order (a wave
// ballot and a prefix over the four waves), so the per-pixel loop runs over
// the few partials above the tile, not over every brick of the frame.
template <int MODE>
__global__ __launch_bounds__(256) void k_over(const PartRect *__restrict__ rects, int32_t n, float *out,
                                              int32_t tile_w, int32_t tile_h) {
    __shared__ PartRect sr[256];
    __shared__ int32_t wn[4];
    const int32_t tid = (int32_t)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t tx0 = blockIdx.x * 16, ty0 = blockIdx.y * 16;
    const int32_t px = tx0 + (tid & 15), py = ty0 + (tid >> 4);
    const bool valid = px < tile_w && py < tile_h;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    float mx = -INFINITY;
    for (int32_t c0 = 0; c0 < n; c0 += 256) {
        const int32_t cn = min(256, n - c0);
        PartRect R{};
        bool hit = false;
        if (tid < cn) {
            R = rects[c0 + tid];
            hit = !(R.x0 > tx0 + 15 || R.y0 > ty0 + 15 || R.x0 + R.w <= tx0 || R.y0 + R.h <= ty0);
        }
        const uint64_t m = __ballot(hit);
        __syncthreads();                    // the previous chunk's readers are done with sr and wn
        if (lane == 0) wn[wv] = __popcll(m);
        __syncthreads();
        int32_t base = 0, total = 0;
#pragma unroll
        for (int32_t k = 0; k < 4; ++k) {
            base += k < wv ? wn[k] : 0;
            total += wn[k];
        }
        if (hit) sr[base + __popcll(m & ((1ull << lane) - 1ull))] = R;
        __syncthreads();
        for (int32_t i = 0; i < total; ++i) {
            const PartRect Q = sr[i];
            if (!valid || px < Q.x0 || py < Q.y0 || px >= Q.x0 + Q.w || py >= Q.y0 + Q.h) continue;
            const int64_t o = (int64_t)(py - Q.y0) * Q.w + (px - Q.x0);
            if (MODE == VR_MIP) {
                mx = fmaxf(mx, Q.data[o]);
            } else {
                const float4 p = ((const float4 *)Q.data)[o];
                const float t = 1.0f - acc.w;
                acc.x = fmaf(t, p.x, acc.x);
                acc.y = fmaf(t, p.y, acc.y);
                acc.z = fmaf(t, p.z, acc.z);
                acc.w = fmaf(t, p.w, acc.w);
            }
        }
    }
    if (!valid) return;
    const int64_t o = (int64_t)py * tile_w + px;
    if (MODE == VR_MIP) out[o] = mx;
    else ((float4 *)out)[o] = acc;
}

template <typename S, int MODE, int FILTER>
static void launch_brick_t(const MarchArgs &a, const BrickJob *jobs, int32_t n, int32_t tiles, hipStream_t s) {
    hipLaunchKernelGGL((k_brick<S, MODE, FILTER>), dim3((unsigned)tiles), dim3(256), 0, s, a, jobs, n);
}

template <typename S>
static void launch_brick_s(const MarchArgs &a, int32_t mode, int32_t filter, const BrickJob *jobs, int32_t n,
                           int32_t tiles, hipStream_t s) {
    if (mode == VR_MIP) {
        if (filter == VR_NEAREST) launch_brick_t<S, VR_MIP, VR_NEAREST>(a, jobs, n, tiles, s);
        else launch_brick_t<S, VR_MIP, VR_TRILINEAR>(a, jobs, n, tiles, s);
    } else {
        if (filter == VR_NEAREST) launch_brick_t<S, VR_COMPOSITE, VR_NEAREST>(a, jobs, n, tiles, s);
        else launch_brick_t<S, VR_COMPOSITE, VR_TRILINEAR>(a, jobs, n, tiles, s);
    }
}

hipError_t launch_bricks(const MarchArgs &a, int32_t mode, int32_t filter, const BrickJob *jobs_dev, int32_t n_jobs,
                         int32_t total_tiles, hipStream_t s) {
    if (n_jobs <= 0 || total_tiles <= 0) return hipSuccess;
    switch (a.vol.dtype) {
        case VR_F32: launch_brick_s<float>(a, mode, filter, jobs_dev, n_jobs, total_tiles, s); break;
        case VR_F16: launch_brick_s<_Float16>(a, mode, filter, jobs_dev, n_jobs, total_tiles, s); break;
        default: launch_brick_s<bf16_t>(a, mode, filter, jobs_dev, n_jobs, total_tiles, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_composite(const PartRect *rects_dev, int32_t n, int32_t mode, float *out, int32_t tile_w,
                            int32_t tile_h, hipStream_t s) {
    dim3 g((unsigned)((tile_w + 15) / 16), (unsigned)((tile_h + 15) / 16)), b(256);
    if (mode == VR_MIP) hipLaunchKernelGGL(k_over<VR_MIP>, g, b, 0, s, rects_dev, n, out, tile_w, tile_h);
    else hipLaunchKernelGGL(k_over<VR_COMPOSITE>, g, b, 0, s, rects_dev, n, out, tile_w, tile_h);
    return hipGetLastError();
}

}  // namespace vr
