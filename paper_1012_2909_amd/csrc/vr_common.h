// vr_common.h -- structures and device helpers shared by the HIP kernels and
// the host runtime of the ray caster.  Geometry conventions are stated in
// include/vr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vr.h"

namespace vr {

// Per-view camera in FP64, basis already computed on the host.
struct CamDev {
    double eye[3], f[3], r[3], u[3];
    double a, b;          // screen half extents: sx = (2(c+1/2)/W - 1) a
    double W, H;          // full frame size
    int32_t kind;         // VR_ORTHO / VR_PERSPECTIVE
    int32_t tile_x0, tile_y0, tile_w, tile_h;
    int32_t pad;
};

// Brick-major volume: bricks of edge B_a along each axis (the whole extent
// when the cube is one brick), each stored as a dense Px*Py*Pz block
// (x fastest) holding voxels [b*B_a - 1, b*B_a + B_a] of the cube, clamped
// to the cube: a one-voxel apron on every side.  The row pitch Px is
// Bx + 2 rounded up to a multiple of 8 elements, so rows start 16-byte
// aligned and 16-byte chunk loads never cross a row; the tail of a row
// repeats the last voxel and is never sampled.
//
// A one-brick layout may hold three copies of the padded cube, each with a
// different fastest axis (copy c stores axis c fastest, then c+1, then c+2,
// cyclically): a renderer reads the copy whose fastest axis runs across its
// ray packets, so neighbouring lanes share cache lines whatever the view.
// data/sx/sy/sz/ori describe the copy a kernel reads; brick layouts have
// one copy, x fastest (sx = 1, sy = Px, sz = Px*Py).
//
// An FP32 three-copy layout also holds a line copy for the object-order MIP:
// each padded row of the x-fastest copy cut into lines of 32 elements, line
// L holding padded x indices [31 L, 31 L + 31] (the last index repeated past
// the row's end), lines of a row consecutive, rows in (z, y) order.  A line is
// one 128-byte cache line, and 31 corner indices with their +1 neighbour fit
// in one line, so a block of 31 corner indices along x reads whole lines.
struct VolDev {
    const void *data;     // element 0 of the copy (or brick array) in use
    int32_t nx, ny, nz;
    int32_t Bx, By, Bz;
    int32_t Px, Py, Pz;   // pitches of the x-fastest copy / of every brick
    int32_t nbx, nby, nbz;
    int32_t dtype;
    int32_t single;       // one brick holds the whole cube
    int64_t brick_elems;  // Px*Py*Pz
    int32_t sx, sy, sz;   // element strides of x, y, z in the copy in use
    int32_t ori;          // fastest axis of the copy in use
    int32_t orients;      // copies stored (1 or 3)
    int32_t pad;
    int64_t copy_off[3];  // element offset of each copy from the layout base
    int64_t line_off;     // element offset of the line copy (FP32 three-copy layouts), else 0
    int32_t lpr;          // lines per padded row of the line copy, 0 when there is none
    int32_t pad2;
    uint32_t *dbg;        // debug builds: device counter of index-range violations (else NULL)
};

// Debug builds (compiled with VR_DEBUG_BOUNDS) check the index range of every
// direct gather and every LDS box read and count violations in the
// context's device counter (VolDev::dbg) instead of trusting the geometry;
// vr_debug_bounds_violations reads the count.  Release builds compile the
// checks away.
#ifdef VR_DEBUG_BOUNDS
#define VR_BOUNDS(v, cond)                                        \
    do {                                                          \
        if (!(cond) && (v).dbg) atomicAdd((v).dbg, 1u);           \
    } while (0)
#else
#define VR_BOUNDS(v, cond) \
    do {                   \
    } while (0)
#endif

// Padded extents of copy c of a one-brick layout: the fastest axis c rounded
// up to a multiple of 8 elements, the other two n + 2.
// Axis a of the cube's extent, by selects (no dynamic indexing of a local
// array, which would put the whole structure in scratch memory).
__host__ __device__ inline int64_t axis_n(const VolDev &v, int a) {
    return a == 0 ? v.nx : (a == 1 ? v.ny : v.nz);
}

__host__ __device__ inline void copy_pitches(const VolDev &v, int c, int64_t &pf, int64_t &pm, int64_t &ps) {
    pf = (axis_n(v, c) + 2 + 7) / 8 * 8;
    pm = axis_n(v, (c + 1) % 3) + 2;
    ps = axis_n(v, (c + 2) % 3) + 2;
}

// Point v (describing copy 0 of a layout) at copy o: base pointer, strides
// and orientation.  No-op for layouts without copies.
__host__ __device__ inline void apply_copy(VolDev &v, int o) {
    if (v.orients < 3 || o <= 0 || o > 2) return;
    int64_t pf, pm, ps;
    copy_pitches(v, o, pf, pm, ps);
    // copy o stores axis o fastest, then o+1, then o+2 (cyclically)
    const int64_t s_o = 1, s_o1 = pf, s_o2 = pf * pm;
    const int64_t off = o == 1 ? v.copy_off[1] : v.copy_off[2];
    v.data = (const char *)v.data + off * (v.dtype == VR_F32 ? 4 : 2);
    // axis a has stride s_o if a == o, s_o1 if a == o+1, s_o2 if a == o+2 (mod 3)
    auto st = [&](int a) { return a == o ? s_o : (a == (o + 1) % 3 ? s_o1 : s_o2); };
    v.sx = (int32_t)st(0);
    v.sy = (int32_t)st(1);
    v.sz = (int32_t)st(2);
    v.ori = o;
}

// The copy whose fastest axis runs along the image rows (largest |r_a|): a
// ray packet spreads mostly along r, so its lanes then share cache lines.
__host__ __device__ inline int best_copy(const double r[3]) {
    int o = 0;
    if (fabs(r[1]) > fabs(r[o])) o = 1;
    if (fabs(r[2]) > fabs(r[o])) o = 2;
    return o;
}

struct LutDev {
    const float4 *rgba;   // n entries, straight RGBA
    int32_t n;
    float vmin;
    float scale;          // (n-1)/(vmax-vmin)
    int32_t pad;
};

// Host-side helper: fill a CamDev from the ABI camera.  Returns false on a
// degenerate basis.
bool make_cam(const vr_camera &c, CamDev *out);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
#define VR_FIX_ONE 4294967296.0   // 2^32: positions are signed 32.32 fixed point

struct Ray {
    double ox, oy, oz;    // origin
    double dx, dy, dz;    // unit direction
    double t0, t1;
    int32_t n;            // samples by definition (0 = miss)
};

// Ray through full-frame pixel (col, row).  Scalars only: arrays written
// through pointers on two branches would not stay in registers.
__host__ __device__ __forceinline__ void cam_ray(const CamDev &c, int col, int row, double &ox, double &oy,
                                                 double &oz, double &dx, double &dy, double &dz) {
    const double sx = (2.0 * (col + 0.5) / c.W - 1.0) * c.a;
    const double sy = (1.0 - 2.0 * (row + 0.5) / c.H) * c.b;
    const bool persp = c.kind == VR_PERSPECTIVE;
    const double x = c.f[0] + sx * c.r[0] + sy * c.u[0];
    const double y = c.f[1] + sx * c.r[1] + sy * c.u[1];
    const double z = c.f[2] + sx * c.r[2] + sy * c.u[2];
    const double nrm = persp ? sqrt(x * x + y * y + z * z) : 1.0;
    dx = persp ? x / nrm : c.f[0];
    dy = persp ? y / nrm : c.f[1];
    dz = persp ? z / nrm : c.f[2];
    ox = persp ? c.eye[0] : c.eye[0] + sx * c.r[0] + sy * c.u[0];
    oy = persp ? c.eye[1] : c.eye[1] + sx * c.r[1] + sy * c.u[1];
    oz = persp ? c.eye[2] : c.eye[2] + sx * c.r[2] + sy * c.u[2];
}

// One axis of the slab test: narrows [a0, a1]; false if the line misses.
__device__ __forceinline__ bool slab_axis(double o, double d, double lo, double hi, double &a0, double &a1) {
    if (d == 0.0) return !(o < lo || o > hi);
    double ta = (lo - o) / d, tb = (hi - o) / d;
    a0 = fmax(a0, fmin(ta, tb));
    a1 = fmin(a1, fmax(ta, tb));
    return true;
}

// Slab interval of the ray's line against the box [lo, hi]; false if it misses.
__device__ __forceinline__ bool slab_box(const Ray &r, double lx, double ly, double lz, double hx, double hy,
                                         double hz, double &tn, double &tf) {
    double a0 = -INFINITY, a1 = INFINITY;
    bool hit = slab_axis(r.ox, r.dx, lx, hx, a0, a1);
    hit = slab_axis(r.oy, r.dy, ly, hy, a0, a1) && hit;
    hit = slab_axis(r.oz, r.dz, lz, hz, a0, a1) && hit;
    tn = a0;
    tf = a1;
    return hit && a0 <= a1;
}

// Number of k >= 0 with t0 + (k + 1/2) step < t1.
__device__ __forceinline__ int32_t sample_count(double t0, double t1, double step) {
    if (!(t1 > t0)) return 0;
    double x = (t1 - t0) / step - 0.5;
    int64_t n = x > 0.0 ? (int64_t)ceil(x) : 0;
    while (n > 0 && t0 + ((double)(n - 1) + 0.5) * step >= t1) --n;
    while (t0 + ((double)n + 0.5) * step < t1) ++n;
    return (int32_t)n;
}

// Ray of a full-frame pixel clipped to the cube.
__device__ __forceinline__ void make_ray(const CamDev &c, const VolDev &v, int col, int row,
                                         double step, Ray &r) {
    cam_ray(c, col, row, r.ox, r.oy, r.oz, r.dx, r.dy, r.dz);
    double tn = 0.0, tf = 0.0;
    const bool hit = slab_box(r, 0.0, 0.0, 0.0, (double)v.nx, (double)v.ny, (double)v.nz, tn, tf);
    r.t0 = hit ? fmax(tn, 0.0) : 0.0;
    r.t1 = hit ? tf : 0.0;
    r.n = hit ? sample_count(r.t0, r.t1, step) : 0;
}

// Fixed-point position of sample k0 (minus `shift`, e.g. 1/2 for the
// trilinear corner grid) and the per-sample increment.
__device__ __forceinline__ void fix_start(const Ray &r, double step, int64_t k0, double shift,
                                          int64_t Q[3], int64_t S[3]) {
    // the position is rounded once; the shift is exact in fixed point, so
    // every kernel sees the same sample positions
    double t = r.t0 + ((double)k0 + 0.5) * step;
    const int64_t sh = __double2ll_rn(shift * VR_FIX_ONE);
    Q[0] = __double2ll_rn((r.ox + t * r.dx) * VR_FIX_ONE) - sh;
    Q[1] = __double2ll_rn((r.oy + t * r.dy) * VR_FIX_ONE) - sh;
    Q[2] = __double2ll_rn((r.oz + t * r.dz) * VR_FIX_ONE) - sh;
    S[0] = __double2ll_rn(step * r.dx * VR_FIX_ONE);
    S[1] = __double2ll_rn(step * r.dy * VR_FIX_ONE);
    S[2] = __double2ll_rn(step * r.dz * VR_FIX_ONE);
}

__device__ __forceinline__ int32_t fix_int(int64_t q) { return (int32_t)(q >> 32); }
__device__ __forceinline__ float fix_frac(int64_t q) {
    return (float)(uint32_t)(q & 0xffffffffu) * 2.3283064365386963e-10f;  // 2^-32
}

// Storage loads widened to FP32.
template <typename S> struct Store;
template <> struct Store<float> {
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
};
struct bf16_t { uint16_t bits; };
template <> struct Store<_Float16> {
    static __device__ __forceinline__ float ld(const _Float16 *p) { return (float)*p; }
};
template <> struct Store<bf16_t> {
    static __device__ __forceinline__ float ld(const bf16_t *p) {
        return __uint_as_float(((uint32_t)p->bits) << 16);
    }
};

// Direct gather from a one-brick (padded) layout through the strides of the
// copy in use: the value at corner-grid index (ix, iy, iz) with fractions f
// (nearest: the voxel at (ix, iy, iz)).
template <typename S, int FILTER>
__device__ __forceinline__ float gsample(const VolDev &v, int32_t ix, int32_t iy, int32_t iz, float fx, float fy,
                                         float fz) {
    const uint32_t sx = (uint32_t)v.sx, sy = (uint32_t)v.sy, sz = (uint32_t)v.sz;
    // padded indices i + 1 (and i + 2 for the trilinear's upper corner) lie in [0, N + 1]
    VR_BOUNDS(v, ix >= -1 && iy >= -1 && iz >= -1 && ix + (FILTER == VR_TRILINEAR) <= v.nx &&
                     iy + (FILTER == VR_TRILINEAR) <= v.ny && iz + (FILTER == VR_TRILINEAR) <= v.nz);
    const S *p = (const S *)v.data + ((uint32_t)(ix + 1) * sx + (uint32_t)(iy + 1) * sy + (uint32_t)(iz + 1) * sz);
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

// Table lookup with linear interpolation; LDS copy of the table.  A NaN
// value (a blank voxel in the sample's footprint) is transparent: its
// opacity is 0, so it adds no colour and leaves the transmittance as it is
// (the clamp already sends NaN to entry 0, so only alpha needs the select).
__device__ __forceinline__ float4 lut_eval(const float4 *L, int n, float vmin, float scale, float s) {
    float x = (s - vmin) * scale;
    x = fminf(fmaxf(x, 0.0f), (float)(n - 1));
    int j = min((int)x, n - 2);
    float w = x - (float)j;
    float4 a = L[j], b = L[j + 1];
    float4 o;
    o.x = fmaf(w, b.x - a.x, a.x);
    o.y = fmaf(w, b.y - a.y, a.y);
    o.z = fmaf(w, b.z - a.z, a.z);
    o.w = s == s ? fmaf(w, b.w - a.w, a.w) : 0.0f;
    return o;
}

// log2(1 - a) for a in [0, 1): hardware log2 of u = 1 - a, with Goldberg's
// correction a / (1 - u) for the rounding of u (exact when u == 1).
__device__ __forceinline__ float log2_one_minus(float a) {
    float u = 1.0f - a;
    if (u == 1.0f) return -a * 1.44269504088896341f;
    return __builtin_amdgcn_logf(u) * (a / (1.0f - u));
}

// Log-space transmittance: L = sum log2(1 - a_k) with a compensated
// (Kahan) sum, T = 2^L.  Its rounding stays near one ulp of T whatever the
// ray length, where the running FP32 product drifts by ~k ulp.
struct LogTrans {
    float L = 0.0f, c = 0.0f;
    __device__ __forceinline__ float step(float a) {
        if (a >= 1.0f) { L = -INFINITY; return 0.0f; }
        if (L == -INFINITY) return 0.0f;
        float y = log2_one_minus(a) - c;
        float t = L + y;
        c = (t - L) - y;
        L = t;
        return __builtin_amdgcn_exp2f(L);
    }
};

// Samples k in [k0, k1) with lo <= P(k) < hi along one axis, P(k) = P0 + k S
// (32.32 fixed point): narrows [k0, k1) to them (empty: k0 > k1 - 1).  The
// brick kernels use it for the exact membership of samples in a brick.
__device__ __forceinline__ void brick_axis_range(int64_t P0, int64_t S, int64_t lo, int64_t hi, int64_t &k0,
                                                 int64_t &k1) {
    auto in = [&](int64_t k) {
        int64_t p = P0 + k * S;
        return p >= lo && p < hi;
    };
    if (S == 0) {
        if (!in(0)) { k0 = 1; k1 = 0; }
        return;
    }
    // first and last k inside, from the FP64 estimate, then exact fix-ups
    double a = ((double)lo - (double)P0) / (double)S, b = ((double)hi - (double)P0) / (double)S;
    double kmin = fmin(a, b), kmax = fmax(a, b);
    int64_t lo_k = (int64_t)fmax(ceil(kmin) - 2.0, (double)k0);
    int64_t hi_k = (int64_t)fmin(floor(kmax) + 2.0, (double)(k1 - 1));
    if (lo_k > hi_k) { k0 = 1; k1 = 0; return; }
    int guard = 0;
    while (lo_k <= hi_k && !in(lo_k) && guard++ < 8) ++lo_k;
    guard = 0;
    while (hi_k >= lo_k && !in(hi_k) && guard++ < 8) --hi_k;
    if (lo_k > hi_k || !in(lo_k) || !in(hi_k)) { k0 = 1; k1 = 0; return; }
    k0 = lo_k;
    k1 = hi_k + 1;
}

// XCD-aware remap: consecutive hardware workgroup ids go round-robin over
// the 8 XCDs; give each XCD a contiguous range of logical ids so that the
// tiles resident on one XCD (sharing its L2) are neighbours.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
    const uint32_t X = 8;
    uint32_t per = nblocks / X;
    uint32_t full = per * X;
    if (bid >= full) return bid;
    return (bid % X) * per + bid / X;
}

// Logical tile of hardware workgroup bid under a tile order (a bijection):
//  0: each XCD takes one contiguous band of tiles (XCD-local L2 reuse);
//  1: hardware order: neighbouring tiles run on different XCDs, so the work
//     of a view whose volume covers only part of the frame spreads evenly;
//  2: blocks of 4 x 4 tiles, each run on one XCD, the blocks dealt over the
//     XCDs in turn: neighbouring tiles share their XCD's L2 (overlapping
//     voxel boxes are fetched once) and the work still spreads evenly;
//  3: the permutation perm (the LDS-staged path's bundles in decreasing
//     order of their estimated box fetch), or order 1 when perm is NULL.
// Workgroups are dealt to the XCDs round-robin by id (bid mod 8), and a
// CU takes the next workgroup as one finishes: with the costliest tiles
// first, the last workgroups to start are short ones.
__device__ __forceinline__ void tile_xy(uint32_t bid, uint32_t nblocks, int32_t gx, int32_t gy, int order,
                                        const int32_t *perm, int32_t &tx, int32_t &ty) {
    if (order == 3) {
        // the tile permutation of the ordering kernel (hardware order without one)
        const uint32_t g = perm ? (uint32_t)perm[bid] : bid;
        tx = (int32_t)(g % (uint32_t)gx);
        ty = (int32_t)(g / (uint32_t)gx);
        return;
    }
    if (order == 2) {
        // enumeration E: strips of 4 tile rows, each walked column by column
        // (16 consecutive E indices form a 4 x 4 block, or a compact block
        // of a shorter last strip)
        const uint32_t X = 8, B = 16, full = nblocks / (X * B) * (X * B);
        uint32_t e = bid;
        if (bid < full) {
            const uint32_t x = bid % X, k = bid / X;
            e = ((k / B) * X + x) * B + k % B;
        }
        const uint32_t strip = e / (4u * (uint32_t)gx);
        const uint32_t h = min(4u, (uint32_t)gy - 4u * strip);
        const uint32_t w = e - strip * 4u * (uint32_t)gx;
        tx = (int32_t)(w / h);
        ty = (int32_t)(4u * strip + w % h);
        return;
    }
    const uint32_t g = order == 1 ? bid : xcd_remap(bid, nblocks);
    tx = (int32_t)(g % (uint32_t)gx);
    ty = (int32_t)(g / (uint32_t)gx);
}

}  // namespace vr
