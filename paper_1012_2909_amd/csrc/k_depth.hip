// k_depth.hip -- per-pixel depth of a render and the catalogue overlay that
// is drawn against it (section 2: the box around each detected source of a
// catalogue is outlined on top of the rendered image and moves with the
// view).
//
// Depth (K9, one-brick layouts): the ray parameter t of one sample per pixel,
//  - composite: the first sample after which the accumulated opacity reaches
//    a level (the same FP32 transmittance arithmetic as the render, so the
//    crossing is the render's own);
//  - MIP: the first sample whose value is the ray's maximum;
// +inf where there is none.  Samples are gathered directly (positions,
// interpolation and table as in every marching kernel).
//
// Overlay (K10): a workgroup owns a 16 x 16 pixel tile.  The boxes are
// culled against the tile in chunks of 256 (one box per thread: the screen
// rectangle of its eight projected corners, or the whole frame when a corner
// lies behind the near plane), the survivors listed in LDS; then every pixel
// tests the 12 edges of each listed box in FP64: the edge, clipped to the
// near plane, is projected to full-frame pixel coordinates; the pixel is
// covered when its centre lies within half_width of the projected segment;
// the edge's depth there is the ray distance of the 3D point under the
// segment's point nearest the centre; the edge is visible when that depth is
// at most the depth image's.  The pixel takes the nearest visible covering
// box (ties: the lower box index) and blends its colour over the image.
#include "vr_internal.h"

namespace vr {

template <typename S, int MODE, int FILTER>
__global__ __launch_bounds__(256) void k_depth(MarchArgs A, float level, float *depth) {
    __shared__ float4 lut[1024];
    if (MODE == VR_COMPOSITE) {
        for (int i = threadIdx.x; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
        __syncthreads();
    }
    const int64_t npix = (int64_t)A.cam.tile_w * A.cam.tile_h;
    const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= npix) return;
    const int32_t px = (int32_t)(pix % A.cam.tile_w), py = (int32_t)(pix / A.cam.tile_w);
    Ray r{};
    make_ray(A.cam, A.vol, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    int64_t Q[3], D[3];
    fix_start(r, A.step, 0, FILTER == VR_TRILINEAR ? 0.5 : 0.0, Q, D);
    int32_t hit = -1;
    if (MODE == VR_MIP) {
        float m = -INFINITY;
        for (int32_t k = 0; k < r.n; ++k) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
            if (FILTER == VR_TRILINEAR) { fx = fix_frac(Q[0]); fy = fix_frac(Q[1]); fz = fix_frac(Q[2]); }
            const float s = gsample<S, FILTER>(A.vol, fix_int(Q[0]), fix_int(Q[1]), fix_int(Q[2]), fx, fy, fz);
            if (s > m) { m = s; hit = k; }          // the first maximum (NaN never wins)
            Q[0] += D[0]; Q[1] += D[1]; Q[2] += D[2];
        }
    } else {
        float T = 1.0f;
        LogTrans lt;
        const bool use_log = A.trans == 1 || (A.trans == 2 && r.n > 1024);
        for (int32_t k = 0; k < r.n; ++k) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
            if (FILTER == VR_TRILINEAR) { fx = fix_frac(Q[0]); fy = fix_frac(Q[1]); fz = fix_frac(Q[2]); }
            const float s = gsample<S, FILTER>(A.vol, fix_int(Q[0]), fix_int(Q[1]), fix_int(Q[2]), fx, fy, fz);
            Q[0] += D[0]; Q[1] += D[1]; Q[2] += D[2];
            const float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
            const float ta = T * c.w;
            T = use_log ? lt.step(c.w) : T - ta;
            if (1.0f - T >= level) { hit = k; break; }
            if (A.ert && T <= A.thr) break;
        }
    }
    depth[pix] = hit >= 0 ? (float)(r.t0 + ((double)hit + 0.5) * A.step) : INFINITY;
}

// ---------------------------------------------------------------------------
// overlay
// ---------------------------------------------------------------------------
// World point -> full-frame pixel coordinates (X, Y) and view depth w along f.
__device__ __forceinline__ void project_px(const CamDev &c, double Px, double Py, double Pz, double &X, double &Y,
                                           double &w) {
    const double d0 = Px - c.eye[0], d1 = Py - c.eye[1], d2 = Pz - c.eye[2];
    const double wf = d0 * c.f[0] + d1 * c.f[1] + d2 * c.f[2];
    const double xr = d0 * c.r[0] + d1 * c.r[1] + d2 * c.r[2];
    const double yu = d0 * c.u[0] + d1 * c.u[1] + d2 * c.u[2];
    const bool persp = c.kind == VR_PERSPECTIVE;
    const double sx = persp ? xr / wf : xr, sy = persp ? yu / wf : yu;
    X = (sx / c.a + 1.0) * 0.5 * c.W;
    Y = (1.0 - sy / c.b) * 0.5 * c.H;
    w = wf;
}

__device__ __forceinline__ double view_w(const CamDev &c, double Px, double Py, double Pz) {
    return (Px - c.eye[0]) * c.f[0] + (Py - c.eye[1]) * c.f[1] + (Pz - c.eye[2]) * c.f[2];
}

// Nearest visible covering edge of box b at pixel centre (qx, qy); +inf if
// none.  Corner coordinates are selected with branches on the edge index
// (no dynamic indexing of a local array).
__device__ double box_depth(const CamDev &c, const vr_box &b, double qx, double qy, double hw, double near,
                            double zb) {
    double best = INFINITY;
    const bool persp = c.kind == VR_PERSPECTIVE;
    for (int e = 0; e < 12; ++e) {
        const int ax = e >> 2;
        // along axis ax from lo to hi; the other two axes take lo or hi by
        // bits 0 and 1 of e (axis ax+1 by bit 0, axis ax+2 by bit 1)
        const bool b1 = e & 1, b2 = e & 2;
        double p0[3], p1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double lo = a == 0 ? b.lo[0] : (a == 1 ? b.lo[1] : b.lo[2]);
            const double hi = a == 0 ? b.hi[0] : (a == 1 ? b.hi[1] : b.hi[2]);
            const int rel = (a - ax + 3) % 3;       // 0: the edge's axis, 1: ax+1, 2: ax+2
            const bool up = rel == 1 ? b1 : b2;
            p0[a] = rel == 0 ? lo : (up ? hi : lo);
            p1[a] = rel == 0 ? hi : (up ? hi : lo);
        }
        if (persp) {
            const double wa = view_w(c, p0[0], p0[1], p0[2]), wb = view_w(c, p1[0], p1[1], p1[2]);
            if (wa < near && wb < near) continue;
            if (wa < near || wb < near) {
                const double t = (near - wa) / (wb - wa);
                const double cx = p0[0] + t * (p1[0] - p0[0]), cy = p0[1] + t * (p1[1] - p0[1]),
                             cz = p0[2] + t * (p1[2] - p0[2]);
                if (wa < near) { p0[0] = cx; p0[1] = cy; p0[2] = cz; }
                else { p1[0] = cx; p1[1] = cy; p1[2] = cz; }
            }
        }
        double X0, Y0, w0, X1, Y1, w1;
        project_px(c, p0[0], p0[1], p0[2], X0, Y0, w0);
        project_px(c, p1[0], p1[1], p1[2], X1, Y1, w1);
        const double dx = X1 - X0, dy = Y1 - Y0, L2 = dx * dx + dy * dy;
        double sp = L2 > 0.0 ? ((qx - X0) * dx + (qy - Y0) * dy) / L2 : 0.0;
        sp = fmin(fmax(sp, 0.0), 1.0);
        const double ex = X0 + sp * dx - qx, ey = Y0 + sp * dy - qy;
        if (sqrt(ex * ex + ey * ey) > hw) continue;
        const double uu = persp ? sp * w0 / (sp * w0 + (1.0 - sp) * w1) : sp;
        const double Px = p0[0] + uu * (p1[0] - p0[0]), Py = p0[1] + uu * (p1[1] - p0[1]),
                     Pz = p0[2] + uu * (p1[2] - p0[2]);
        double t;
        if (persp) {
            const double d0 = Px - c.eye[0], d1 = Py - c.eye[1], d2 = Pz - c.eye[2];
            t = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        } else {
            t = view_w(c, Px, Py, Pz);
        }
        if (!(t <= zb)) continue;
        best = fmin(best, t);
    }
    return best;
}

// Conservative screen rectangle of box b (full-frame pixel coordinates);
// false when the whole box lies behind the near plane.
__device__ bool box_rect(const CamDev &c, const vr_box &b, double near, double &x0, double &y0, double &x1,
                         double &y1) {
    x0 = y0 = INFINITY;
    x1 = y1 = -INFINITY;
    bool behind = false, front = false;
    for (int k = 0; k < 8; ++k) {
        const double Px = (k & 1) ? b.hi[0] : b.lo[0], Py = (k & 2) ? b.hi[1] : b.lo[1],
                     Pz = (k & 4) ? b.hi[2] : b.lo[2];
        double X, Y, w;
        project_px(c, Px, Py, Pz, X, Y, w);
        if (c.kind == VR_PERSPECTIVE && w < near) { behind = true; continue; }
        front = true;
        x0 = fmin(x0, X); x1 = fmax(x1, X); y0 = fmin(y0, Y); y1 = fmax(y1, Y);
    }
    if (!front) return false;
    if (behind || !(x1 - x0 < 1e9) || !(y1 - y0 < 1e9)) {   // clipped edges can reach anywhere
        x0 = y0 = -INFINITY;
        x1 = y1 = INFINITY;
    }
    return true;
}

__global__ __launch_bounds__(256) void k_overlay(CamDev cam, const vr_box *boxes, int32_t n, double hw, double near,
                                                 const float *depth, float4 *img, int32_t tiles_x) {
    __shared__ vr_box list[256];
    __shared__ int32_t idx[256];
    __shared__ int32_t count;
    const int32_t tx = (int32_t)(blockIdx.x % (uint32_t)tiles_x), ty = (int32_t)(blockIdx.x / (uint32_t)tiles_x);
    const int32_t px = tx * 16 + (int32_t)(threadIdx.x & 15), py = ty * 16 + (int32_t)(threadIdx.x >> 4);
    const bool valid = px < cam.tile_w && py < cam.tile_h;
    const double qx = cam.tile_x0 + px + 0.5, qy = cam.tile_y0 + py + 0.5;
    // the tile in full-frame pixel coordinates, widened by the half width
    // (and a margin far above the rounding of the projections)
    const double hm = hw + 1e-6;
    const double rx0 = cam.tile_x0 + tx * 16 - hm, rx1 = cam.tile_x0 + tx * 16 + 16 + hm;
    const double ry0 = cam.tile_y0 + ty * 16 - hm, ry1 = cam.tile_y0 + ty * 16 + 16 + hm;
    const int64_t pix = (int64_t)py * cam.tile_w + px;
    const double zb = (valid && depth) ? (double)depth[pix] : INFINITY;
    double best = INFINITY;
    int32_t best_i = -1;
    float4 col = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int32_t c0 = 0; c0 < n; c0 += 256) {
        if (threadIdx.x == 0) count = 0;
        __syncthreads();
        const int32_t i = c0 + (int32_t)threadIdx.x;
        if (i < n) {
            const vr_box b = boxes[i];
            double x0, y0, x1, y1;
            if (box_rect(cam, b, near, x0, y0, x1, y1) && x1 >= rx0 && x0 <= rx1 && y1 >= ry0 && y0 <= ry1) {
                const int32_t slot = atomicAdd(&count, 1);
                list[slot] = b;
                idx[slot] = i;
            }
        }
        __syncthreads();
        const int32_t m = count;
        if (valid) {
            for (int32_t j = 0; j < m; ++j) {
                const double t = box_depth(cam, list[j], qx, qy, hw, near, zb);
                // nearest box, ties to the lower index (the list order is not fixed)
                if (t < best || (t == best && t < INFINITY && idx[j] < best_i)) {
                    best = t;
                    best_i = idx[j];
                    col = make_float4(list[j].rgba[0], list[j].rgba[1], list[j].rgba[2], list[j].rgba[3]);
                }
            }
        }
        __syncthreads();
    }
    if (valid && best_i >= 0) {
        float4 o = img[pix];
        const float a = col.w, k = 1.0f - a;
        o.x = col.x * a + k * o.x;
        o.y = col.y * a + k * o.y;
        o.z = col.z * a + k * o.z;
        o.w = a + k * o.w;
        img[pix] = o;
    }
}

template <typename S, int MODE>
static hipError_t launch_depth_m(const MarchArgs &a, int32_t filter, float level, float *depth, hipStream_t s) {
    const int64_t npix = (int64_t)a.cam.tile_w * a.cam.tile_h;
    dim3 g((unsigned)((npix + 255) / 256)), b(256);
    if (filter == VR_NEAREST) hipLaunchKernelGGL((k_depth<S, MODE, VR_NEAREST>), g, b, 0, s, a, level, depth);
    else hipLaunchKernelGGL((k_depth<S, MODE, VR_TRILINEAR>), g, b, 0, s, a, level, depth);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_depth_s(const MarchArgs &a, int32_t mode, int32_t filter, float level, float *depth,
                                 hipStream_t s) {
    return mode == VR_MIP ? launch_depth_m<S, VR_MIP>(a, filter, level, depth, s)
                          : launch_depth_m<S, VR_COMPOSITE>(a, filter, level, depth, s);
}

hipError_t launch_depth(const MarchArgs &a, int32_t mode, int32_t filter, float level, float *depth, hipStream_t s) {
    if ((int64_t)a.cam.tile_w * a.cam.tile_h == 0) return hipSuccess;
    switch (a.vol.dtype) {
        case VR_F32: return launch_depth_s<float>(a, mode, filter, level, depth, s);
        case VR_F16: return launch_depth_s<_Float16>(a, mode, filter, level, depth, s);
        default: return launch_depth_s<bf16_t>(a, mode, filter, level, depth, s);
    }
}

hipError_t launch_overlay(const CamDev &cam, const vr_box *boxes, int32_t n, double hw, double near,
                          const float *depth, float *img, hipStream_t s) {
    if (n <= 0 || (int64_t)cam.tile_w * cam.tile_h == 0) return hipSuccess;
    const int32_t tiles_x = (cam.tile_w + 15) / 16, tiles_y = (cam.tile_h + 15) / 16;
    hipLaunchKernelGGL(k_overlay, dim3((unsigned)(tiles_x * tiles_y)), dim3(256), 0, s, cam, boxes, n, hw, near,
                       depth, (float4 *)img, tiles_x);
    return hipGetLastError();
}

}  // namespace vr
