// k_slab.hip -- K1/K2 with LDS-staged voxel boxes: the headline renderer.
//
// A workgroup owns a bundle of bw x bh neighbouring pixels (one ray per
// lane).  The bundle marches through the cube in slabs perpendicular to its
// dominant axis w: slab c holds the samples whose trilinear corner index
// along w lies in [cL, cL+L).  For each slab the workgroup computes the voxel
// box all of its samples can touch (from the bundle's four corner rays: the
// rays through the bundle's pixels fill the convex frustum they span), copies
// that box from HBM into LDS with aligned 16-byte loads (x is the storage
// order), and then every lane walks its own samples of the slab reading the 8
// corners from LDS.  Samples of one ray are visited in order, slab after
// slab, so the composite stays front to back.  Every voxel box is read from
// HBM once per bundle instead of being gathered corner by corner.
//
// Arithmetic is the same as k_march: FP64 ray set-up, 32.32 fixed-point
// positions advanced by an exact integer step, FP32 sampling / table /
// compositing, so the two paths give identical images.  Lanes whose ray does
// not run along the bundle's slab direction, and slabs whose box does not fit
// the LDS budget, fall back to direct gathers.  Single-brick layouts only.
#include "vr_internal.h"

namespace vr {

struct SlabArgs {
    MarchArgs m;
    int32_t bw, bh;       // bundle in pixels (bw*bh = threads per workgroup)
    int32_t cap;          // LDS box capacity in floats
    int32_t lmax;         // largest slab thickness tried
};

// Sample from the LDS box at element offset off; lsx/lsy/lsz are the box
// strides of x, y and z (the box keeps the axis order of the copy it came
// from).
template <int FILTER>
__device__ __forceinline__ float lsample(const float *box, uint32_t off, uint32_t lsx, uint32_t lsy, uint32_t lsz,
                                         float fx, float fy, float fz) {
    if (FILTER == VR_NEAREST) return box[off];
    const float *p = box + off;
    float c000 = p[0], c100 = p[lsx], c010 = p[lsy], c110 = p[lsy + lsx];
    const float *q = p + lsz;
    float c001 = q[0], c101 = q[lsx], c011 = q[lsy], c111 = q[lsy + lsx];
    float x00 = fmaf(fx, c100 - c000, c000), x10 = fmaf(fx, c110 - c010, c010);
    float x01 = fmaf(fx, c101 - c001, c001), x11 = fmaf(fx, c111 - c011, c011);
    float y0 = fmaf(fy, x10 - x00, x00), y1 = fmaf(fy, x11 - x01, x01);
    return fmaf(fz, y1 - y0, y0);
}

// 16 bytes of storage -> floats in LDS.
__device__ __forceinline__ void put_chunk(float *dst, const float *src) {
    *(float4 *)dst = *(const float4 *)src;
}
__device__ __forceinline__ void put_chunk(float *dst, const _Float16 *src) {
    typedef _Float16 h8 __attribute__((ext_vector_type(8)));
    h8 v = *(const h8 *)src;
    *(float4 *)dst = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    *(float4 *)(dst + 4) = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
}
__device__ __forceinline__ void put_chunk(float *dst, const bf16_t *src) {
    uint4 v = *(const uint4 *)src;
    *(float4 *)dst = make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                                 __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
    *(float4 *)(dst + 4) = make_float4(__uint_as_float(v.z << 16), __uint_as_float(v.z & 0xffff0000u),
                                       __uint_as_float(v.w << 16), __uint_as_float(v.w & 0xffff0000u));
}

__device__ __forceinline__ int32_t wave_min(int32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Workgroup min/max through a small LDS scratch (two barriers).
__device__ __forceinline__ void wg_minmax(int32_t &mn, int32_t &mx, int32_t *red) {
    int32_t a = wave_min(mn), b = wave_max(mx);
    int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[w] = a; red[8 + w] = b; }
    __syncthreads();
    mn = red[0];
    mx = red[8];
    for (int i = 1; i < nw; ++i) { mn = min(mn, red[i]); mx = max(mx, red[8 + i]); }
}

// Floor division for possibly negative numerators (positive divisor).
__device__ __forceinline__ int32_t fdiv(int32_t a, int32_t b) {
    int32_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

// Uniform description of the bundle's frustum: per corner ray the lateral
// coordinates along axes u, v as affine functions of the position along w.
struct Frustum {
    float au[4], bu[4], av[4], bv[4];
    int32_t Nu, Nv, Nw;
    float h;              // 1/2 for the trilinear corner grid, 0 for nearest
};

// Corner-index box of the samples whose corner index along w lies in
// [lo_w, lo_w + L): lateral from the corner rays at both slab faces (plus a
// margin above FP32 rounding), clipped to the padded cube [-1, N].
__device__ __forceinline__ void slab_box(const Frustum &F, int32_t lo_w, int32_t L, int32_t &lu, int32_t &hu,
                                         int32_t &lv, int32_t &hv, int32_t &lw, int32_t &hw) {
    const float p0 = (float)lo_w + F.h, p1 = (float)(lo_w + L) + F.h;
    float mnu = 3e38f, mxu = -3e38f, mnv = 3e38f, mxv = -3e38f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float u0 = fmaf(F.bu[c], p0, F.au[c]), u1 = fmaf(F.bu[c], p1, F.au[c]);
        float v0 = fmaf(F.bv[c], p0, F.av[c]), v1 = fmaf(F.bv[c], p1, F.av[c]);
        mnu = fminf(mnu, fminf(u0, u1)); mxu = fmaxf(mxu, fmaxf(u0, u1));
        mnv = fminf(mnv, fminf(v0, v1)); mxv = fmaxf(mxv, fmaxf(v0, v1));
    }
    const float big = 1e8f, marg = 0.02f;
    mnu = fminf(fmaxf(mnu - F.h - marg, -big), big); mxu = fminf(fmaxf(mxu - F.h + marg, -big), big);
    mnv = fminf(fmaxf(mnv - F.h - marg, -big), big); mxv = fminf(fmaxf(mxv - F.h + marg, -big), big);
    lu = max((int32_t)floorf(mnu), -1);
    hu = min((int32_t)floorf(mxu) + 1, F.Nu);
    lv = max((int32_t)floorf(mnv), -1);
    hv = min((int32_t)floorf(mxv) + 1, F.Nv);
    lw = max(lo_w, -1);
    hw = min(lo_w + L, F.Nw);
}

// Dimensions of the LDS copy of a box along the copy's fastest axis (in
// padded-layout index, widened to whole 16-byte chunks of EPC elements) and
// along its two other axes.
template <int EPC>
__device__ __forceinline__ void box_dims(int32_t f0, int32_t f1, int32_t m0, int32_t m1, int32_t s0, int32_t s1,
                                         int32_t &fp0, int32_t &Df, int32_t &Dm, int32_t &Ds) {
    fp0 = ((f0 + 1) / EPC) * EPC;
    const int32_t fp1 = f1 + 1;
    Df = fp1 < fp0 ? 0 : ((fp1 - fp0 + 1) + EPC - 1) / EPC * EPC;
    Dm = max(m1 - m0 + 1, 0);
    Ds = max(s1 - s0 + 1, 0);
}

// Per-lane marching state.
struct LaneState {
    int64_t Q[3], D[3];
    int32_t n, k;
    float m, T, C0, C1, C2;
    LogTrans lt;
    bool use_log, stopped;
};

template <int MODE>
__device__ __forceinline__ bool consume(LaneState &L, const MarchArgs &A, const float4 *lut, int64_t pix,
                                        int64_t npix, float s) {
    if (MODE == VR_MIP) {
        L.m = fmaxf(L.m, s);
        return true;
    }
    if (A.ckpt && (L.k & 63) == 0 && (L.k >> 6) < A.ckpt_segs) A.ckpt[(int64_t)(L.k >> 6) * npix + pix] = L.T;
    float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
    float ta = L.T * c.w;
    L.C0 = fmaf(ta, c.x, L.C0);
    L.C1 = fmaf(ta, c.y, L.C1);
    L.C2 = fmaf(ta, c.z, L.C2);
    L.T = L.use_log ? L.lt.step(c.w) : L.T - ta;
    return !(A.ert && L.T <= A.thr);
}

// The slab march for slab axis W (0, 1, 2 = x, y, z) over the copy whose
// fastest axis is ORI.
template <typename S, int MODE, int FILTER, int W, int ORI>
__device__ __forceinline__ void run_slabs(const SlabArgs &SA, const Frustum &F, LaneState &ls, bool active,
                                          int32_t L, int32_t sw, int32_t c, float *box, const float4 *lut,
                                          int64_t pix, int64_t npix) {
    const MarchArgs &A = SA.m;
    const VolDev &V = A.vol;
    constexpr int U = W == 0 ? 1 : 0, VV = W == 2 ? 1 : 2;
    constexpr int AF = ORI, AM = (ORI + 1) % 3, AS = (ORI + 2) % 3;   // fastest, middle, slowest axis
    constexpr int EPC = 16 / (int)sizeof(S);          // storage elements per 16-byte chunk
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int32_t max_iter = (F.Nw + 2) / L + 3;
    const uint32_t gstr[3] = {(uint32_t)V.sx, (uint32_t)V.sy, (uint32_t)V.sz};
    int32_t iter = 0;
    while (__syncthreads_or(active) && iter++ < max_iter) {
        const int32_t lo_w = c * L;
        int32_t lu, hu, lv, hv, lw, hw;
        slab_box(F, lo_w, L, lu, hu, lv, hv, lw, hw);
        int32_t b0[3], b1[3];
        b0[W] = lw; b1[W] = hw; b0[U] = lu; b1[U] = hu; b0[VV] = lv; b1[VV] = hv;
        int32_t fp0, Df, Dm, Ds;
        box_dims<EPC>(b0[AF], b1[AF], b0[AM], b1[AM], b0[AS], b1[AS], fp0, Df, Dm, Ds);
        const bool empty = Df <= 0 || Dm <= 0 || Ds <= 0;
        const bool fits = FILTER == VR_NEAREST || (Df >= 2 && Dm >= 2 && Ds >= 2);
        const bool use_lds = !empty && fits && (int64_t)Df * Dm * Ds <= SA.cap;
        if (use_lds) {
            // chunks per row, lanes per row (power of two), rows per pass
            const int32_t cpr = Df / EPC;
            int32_t lpr = 1;
            while (lpr < cpr && lpr < nthr) lpr <<= 1;
            const int32_t rpp = nthr / lpr;
            const int32_t tx = tid % lpr;
            int32_t row = tid / lpr;
            int32_t mm = row % Dm, ss = row / Dm;           // once per slab
            const int32_t mstep = rpp % Dm, sstep = rpp / Dm;
            const int32_t rows = Dm * Ds;
            for (; row < rows; row += rpp) {
                const S *src = (const S *)V.data + ((size_t)(b0[AS] + ss + 1) * gstr[AS] +
                                                    (size_t)(b0[AM] + mm + 1) * gstr[AM] + (size_t)fp0);
                float *dst = box + (size_t)row * Df;
                for (int32_t cx = tx; cx < cpr; cx += lpr) put_chunk(dst + cx * EPC, src + cx * EPC);
                mm += mstep;
                ss += sstep;
                if (mm >= Dm) { mm -= Dm; ++ss; }
            }
            __syncthreads();
        }
        if (active) {
            // box strides of x, y, z and the box origin in padded index
            uint32_t lstr[3];
            lstr[AF] = 1;
            lstr[AM] = (uint32_t)Df;
            lstr[AS] = (uint32_t)Df * (uint32_t)Dm;
            int32_t org[3], lim[3];
            org[AF] = fp0 - 1; org[AM] = b0[AM]; org[AS] = b0[AS];
            const int32_t t1 = FILTER == VR_TRILINEAR ? 1 : 0;
            lim[AF] = Df - 1 - t1; lim[AM] = Dm - 1 - t1; lim[AS] = Ds - 1 - t1;
            const int32_t wlast = lo_w + L - 1;
            while (true) {
                const int32_t iw = fix_int(ls.Q[W]);
                if (sw > 0 ? iw > wlast : iw < lo_w) break;           // left the slab
                const int32_t ix = fix_int(ls.Q[0]), iy = fix_int(ls.Q[1]), iz = fix_int(ls.Q[2]);
                float fx = 0.f, fy = 0.f, fz = 0.f;
                if (FILTER == VR_TRILINEAR) { fx = fix_frac(ls.Q[0]); fy = fix_frac(ls.Q[1]); fz = fix_frac(ls.Q[2]); }
                float s;
                if (use_lds) {
                    // the clamp keeps every read inside the box
                    const uint32_t lx = (uint32_t)min(max(ix - org[0], 0), lim[0]);
                    const uint32_t ly = (uint32_t)min(max(iy - org[1], 0), lim[1]);
                    const uint32_t lz = (uint32_t)min(max(iz - org[2], 0), lim[2]);
                    s = lsample<FILTER>(box, lx * lstr[0] + ly * lstr[1] + lz * lstr[2], lstr[0], lstr[1], lstr[2],
                                        fx, fy, fz);
                } else {
                    s = gsample<S, FILTER>(V, ix, iy, iz, fx, fy, fz);
                }
                ls.Q[0] += ls.D[0]; ls.Q[1] += ls.D[1]; ls.Q[2] += ls.D[2];
                const bool go = consume<MODE>(ls, A, lut, pix, npix, s);
                ++ls.k;
                if (!go) { ls.stopped = true; active = false; break; }
                if (ls.k >= ls.n) { active = false; break; }
            }
        }
        c += sw;
    }
}

// One bundle of bw x bh pixels whose top-left pixel is (bx0, by0) of the
// viewport in SA.m (called by every thread of the workgroup).  smem holds the
// table (composite) followed by the voxel box; red is a 16-int scratch.
template <typename S, int MODE, int FILTER, int ORI>
__device__ __forceinline__ void slab_bundle(const SlabArgs &SA, int bx0, int by0, float *smem, int32_t *red) {
    const MarchArgs &A = SA.m;
    const int tid = threadIdx.x;
    float4 *lut = (float4 *)smem;                               // composite: n entries
    float *box = smem + (MODE == VR_COMPOSITE ? 4 * A.lut.n : 0);
    const int px = bx0 + tid % SA.bw, py = by0 + tid / SA.bw;
    const bool valid = px < A.cam.tile_w && py < A.cam.tile_h;
    const VolDev &V = A.vol;
    const double h = FILTER == VR_TRILINEAR ? 0.5 : 0.0;

    Ray r{};
    if (valid) make_ray(A.cam, V, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    LaneState ls;
    fix_start(r, A.step, 0, h, ls.Q, ls.D);
    ls.n = r.n;
    ls.k = 0;
    ls.m = -INFINITY;
    ls.T = 1.0f;
    ls.C0 = ls.C1 = ls.C2 = 0.0f;
    ls.use_log = (MODE == VR_COMPOSITE) && (A.trans == 1 || (A.trans == 2 && r.n > 1024));
    ls.stopped = false;

    // ---- the bundle's slab axis and corner rays (uniform) -----------------
    const int cx1 = min(bx0 + SA.bw, A.cam.tile_w) - 1, cy1 = min(by0 + SA.bh, A.cam.tile_h) - 1;
    double cox[4], coy[4], coz[4], cdx[4], cdy[4], cdz[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        cam_ray(A.cam, A.cam.tile_x0 + ((c & 1) ? cx1 : bx0), A.cam.tile_y0 + ((c & 2) ? cy1 : by0), cox[c], coy[c],
                coz[c], cdx[c], cdy[c], cdz[c]);
    const double dcx = cdx[0] + cdx[1] + cdx[2] + cdx[3];
    const double dcy = cdy[0] + cdy[1] + cdy[2] + cdy[3];
    const double dcz = cdz[0] + cdz[1] + cdz[2] + cdz[3];
    int w = 0;
    if (fabs(dcy) > fabs(dcx)) w = 1;
    if (fabs(dcz) > fabs(w == 1 ? dcy : dcx)) w = 2;
    const double dcw = w == 0 ? dcx : (w == 1 ? dcy : dcz);
    const int sw = dcw > 0 ? 1 : -1;
    const int u = w == 0 ? 1 : 0, v2 = w == 2 ? 1 : 2;
    auto pick = [](double x, double y, double z, int ax) -> double { return ax == 0 ? x : (ax == 1 ? y : z); };
    Frustum F;
    bool bundle_ok = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double dw = pick(cdx[c], cdy[c], cdz[c], w);
        if (!(dw * sw >= 0.2)) bundle_ok = false;
        const double ow = pick(cox[c], coy[c], coz[c], w);
        const double su = pick(cdx[c], cdy[c], cdz[c], u) / dw, sv = pick(cdx[c], cdy[c], cdz[c], v2) / dw;
        F.bu[c] = (float)su;
        F.au[c] = (float)(pick(cox[c], coy[c], coz[c], u) - ow * su);
        F.bv[c] = (float)sv;
        F.av[c] = (float)(pick(cox[c], coy[c], coz[c], v2) - ow * sv);
    }
    const int32_t N[3] = {V.nx, V.ny, V.nz};
    F.Nw = w == 0 ? N[0] : (w == 1 ? N[1] : N[2]);
    F.Nu = u == 0 ? N[0] : N[1];
    F.Nv = v2 == 1 ? N[1] : N[2];
    F.h = (float)h;
    const int64_t Qw0 = w == 0 ? ls.Q[0] : (w == 1 ? ls.Q[1] : ls.Q[2]);
    const int64_t Dw = w == 0 ? ls.D[0] : (w == 1 ? ls.D[1] : ls.D[2]);
    const double rdw = w == 0 ? r.dx : (w == 1 ? r.dy : r.dz);
    const bool reg = r.n > 0 && bundle_ok && (Dw > 0) == (sw > 0) && fabs(rdw) >= 0.2;

    // corner-index range along w of all regular lanes
    int32_t wlo, whi;
    {
        const int32_t first = fix_int(Qw0), last = fix_int(Qw0 + (int64_t)(r.n > 0 ? r.n - 1 : 0) * Dw);
        int32_t a = reg ? min(first, last) : INT32_MAX, b = reg ? max(first, last) : INT32_MIN;
        wg_minmax(a, b, red);
        wlo = a;
        whi = b;
    }
    // slab thickness: the largest L whose boxes at both ends of the
    // traversal fit the budget (a perspective bundle widens with depth)
    int32_t L = 0;
    if (wlo <= whi && bundle_ok) {
        for (int32_t cand = SA.lmax; cand >= 1; cand = (cand > 8 ? cand - 4 : cand - 1)) {
            int64_t e[2];
#pragma unroll
            for (int end = 0; end < 2; ++end) {
                const int32_t lo = (end == 0) == (sw > 0) ? whi - cand + 1 : wlo;
                int32_t lu, hu, lv, hv, lw, hw;
                slab_box(F, lo, cand, lu, hu, lv, hv, lw, hw);
                int32_t q0[3], q1[3];
                q0[0] = w == 0 ? lw : lu; q1[0] = w == 0 ? hw : hu;
                q0[1] = w == 0 ? lu : (w == 1 ? lw : lv); q1[1] = w == 0 ? hu : (w == 1 ? hw : hv);
                q0[2] = w == 2 ? lw : lv; q1[2] = w == 2 ? hw : hv;
                constexpr int AF = ORI, AM = (ORI + 1) % 3, AS = (ORI + 2) % 3;
                constexpr int EPC = 16 / (int)sizeof(S);
                int32_t fp0, Df, Dm, Ds;
                // the chunk origin shifts from slab to slab: allow for the widest alignment
                box_dims<EPC>(q0[AF], q1[AF] + EPC - 1, q0[AM], q1[AM], q0[AS], q1[AS], fp0, Df, Dm, Ds);
                e[end] = (int64_t)Df * Dm * Ds;
            }
            if (max(e[0], e[1]) <= SA.cap) { L = cand; break; }
        }
    }

    if (MODE == VR_COMPOSITE) {   // table to LDS (after the FP64 set-up)
        for (int i = tid; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
        __syncthreads();
    }
    const int64_t npix = (int64_t)A.cam.tile_w * A.cam.tile_h;
    const int64_t pix = (int64_t)py * A.cam.tile_w + px;

    if (L > 0) {
        const bool active = reg;
        const int32_t c0 = sw > 0 ? fdiv(wlo, L) : fdiv(whi, L);
        if (w == 0) run_slabs<S, MODE, FILTER, 0, ORI>(SA, F, ls, active, L, sw, c0, box, lut, pix, npix);
        else if (w == 1) run_slabs<S, MODE, FILTER, 1, ORI>(SA, F, ls, active, L, sw, c0, box, lut, pix, npix);
        else run_slabs<S, MODE, FILTER, 2, ORI>(SA, F, ls, active, L, sw, c0, box, lut, pix, npix);
    }
    // lanes outside the slab scheme (and any samples left over) march on
    // with direct gathers
    if (valid && !ls.stopped && ls.k < ls.n) {
        while (ls.k < ls.n) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
            if (FILTER == VR_TRILINEAR) { fx = fix_frac(ls.Q[0]); fy = fix_frac(ls.Q[1]); fz = fix_frac(ls.Q[2]); }
            float s = gsample<S, FILTER>(V, fix_int(ls.Q[0]), fix_int(ls.Q[1]), fix_int(ls.Q[2]), fx, fy, fz);
            ls.Q[0] += ls.D[0]; ls.Q[1] += ls.D[1]; ls.Q[2] += ls.D[2];
            const bool go = consume<MODE>(ls, A, lut, pix, npix, s);
            ++ls.k;
            if (!go) break;
        }
    }
    if (valid) {
        if (A.out) {
            if (MODE == VR_MIP) ((float *)A.out)[pix] = ls.m;
            else ((float4 *)A.out)[pix] = make_float4(ls.C0, ls.C1, ls.C2, 1.0f - ls.T);
        }
        if (A.counts) A.counts[pix] = ls.k;
        if (A.taken) A.taken[pix] = ls.k;
    }
}

template <typename S, int MODE, int FILTER, int ORI>
__global__ __launch_bounds__(256) void k_slab(SlabArgs SA) {
    extern __shared__ float smem[];
    __shared__ int32_t red[16];
    const uint32_t group = tile_order(blockIdx.x, gridDim.x, SA.m.order);
    const int gbx = group % SA.m.groups_x, gby = group / SA.m.groups_x;
    slab_bundle<S, MODE, FILTER, ORI>(SA, gbx * SA.bw, gby * SA.bh, smem, red);
}

// K6: persistent workgroups pull bundles from an atomic queue until every
// bundle of every view is done (each workgroup exits once the counter passes
// the item count).  Items are numbered view by view, largest views first.
template <typename S, int MODE, int FILTER>
__global__ __launch_bounds__(256) void k_batch(BatchArgs B) {
    extern __shared__ float smem[];
    __shared__ int32_t red[16];
    __shared__ int32_t item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = (int32_t)atomicAdd(B.queue, 1u);
        __syncthreads();
        const int32_t item = item_s;
        __syncthreads();
        if (item >= B.total_items) break;
        int32_t lo = 0, hi = B.n_views - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (B.views[mid].tile_begin <= item) lo = mid;
            else hi = mid - 1;
        }
        const ViewDev &V = B.views[lo];
        SlabArgs SA{};
        SA.m.cam = V.cam;
        SA.m.vol = B.vol;
        apply_copy(SA.m.vol, V.ori);
        SA.m.lut.rgba = B.luts + (int64_t)V.lut_index * B.lut_n;
        SA.m.lut.n = B.lut_n;
        SA.m.lut.vmin = B.vmin;
        SA.m.lut.scale = B.scale;
        SA.m.step = B.step;
        SA.m.thr = B.thr;
        SA.m.ert = B.ert;
        SA.m.trans = B.trans;
        SA.m.out = V.out;
        SA.m.groups_x = V.tiles_x;
        SA.bw = B.bw;
        SA.bh = B.bh;
        SA.cap = B.cap;
        SA.lmax = B.lmax;
        const int32_t t = item - V.tile_begin;
        const int bx0 = (t % V.tiles_x) * B.bw, by0 = (t / V.tiles_x) * B.bh;
        if (V.ori == 1) slab_bundle<S, MODE, FILTER, 1>(SA, bx0, by0, smem, red);
        else if (V.ori == 2) slab_bundle<S, MODE, FILTER, 2>(SA, bx0, by0, smem, red);
        else slab_bundle<S, MODE, FILTER, 0>(SA, bx0, by0, smem, red);
        __syncthreads();   // the table and box in LDS are rewritten by the next item
    }
}

__global__ void k_reset_u32(uint32_t *p, int32_t n) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_reset_u32(uint32_t *p, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename S, int MODE, int FILTER>
static hipError_t launch_batch_t(const BatchArgs &a, int32_t groups, hipStream_t s) {
    const size_t lds = (size_t)a.cap * 4 + (MODE == VR_COMPOSITE ? (size_t)a.lut_n * 16 : 0);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_batch<S, MODE, FILTER>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_batch<S, MODE, FILTER>), dim3((unsigned)groups), dim3((unsigned)(a.bw * a.bh)), lds, s, a);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_batch_s(const BatchArgs &a, int32_t mode, int32_t filter, int32_t groups, hipStream_t s) {
    if (mode == VR_MIP) {
        if (filter == VR_NEAREST) return launch_batch_t<S, VR_MIP, VR_NEAREST>(a, groups, s);
        return launch_batch_t<S, VR_MIP, VR_TRILINEAR>(a, groups, s);
    }
    if (filter == VR_NEAREST) return launch_batch_t<S, VR_COMPOSITE, VR_NEAREST>(a, groups, s);
    return launch_batch_t<S, VR_COMPOSITE, VR_TRILINEAR>(a, groups, s);
}

hipError_t launch_batch(const BatchArgs &a, int32_t mode, int32_t filter, int32_t groups, hipStream_t s) {
    if (groups <= 0 || a.total_items <= 0) return hipSuccess;
    switch (a.vol.dtype) {
        case VR_F32: return launch_batch_s<float>(a, mode, filter, groups, s);
        case VR_F16: return launch_batch_s<_Float16>(a, mode, filter, groups, s);
        default: return launch_batch_s<bf16_t>(a, mode, filter, groups, s);
    }
}

template <typename S, int MODE, int FILTER, int ORI>
static hipError_t launch_slab_o(const SlabArgs &a, dim3 g, dim3 b, size_t lds, hipStream_t s) {
    // dynamic LDS beyond 64 KiB needs an explicit opt-in of the exact size
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_slab<S, MODE, FILTER, ORI>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_slab<S, MODE, FILTER, ORI>), g, b, lds, s, a);
    return hipGetLastError();
}

template <typename S, int MODE, int FILTER>
static hipError_t launch_slab_t(const SlabArgs &a, dim3 g, dim3 b, size_t lds, hipStream_t s) {
    switch (a.m.vol.ori) {
        case 0: return launch_slab_o<S, MODE, FILTER, 0>(a, g, b, lds, s);
        case 1: return launch_slab_o<S, MODE, FILTER, 1>(a, g, b, lds, s);
        default: return launch_slab_o<S, MODE, FILTER, 2>(a, g, b, lds, s);
    }
}

template <typename S>
static hipError_t launch_slab_s(const SlabArgs &a, int32_t mode, int32_t filter, dim3 g, dim3 b, size_t lds,
                                hipStream_t s) {
    if (mode == VR_MIP) {
        if (filter == VR_NEAREST) return launch_slab_t<S, VR_MIP, VR_NEAREST>(a, g, b, lds, s);
        return launch_slab_t<S, VR_MIP, VR_TRILINEAR>(a, g, b, lds, s);
    }
    if (filter == VR_NEAREST) return launch_slab_t<S, VR_COMPOSITE, VR_NEAREST>(a, g, b, lds, s);
    return launch_slab_t<S, VR_COMPOSITE, VR_TRILINEAR>(a, g, b, lds, s);
}

hipError_t launch_slab(const MarchArgs &m, int32_t mode, int32_t filter, int32_t bw, int32_t bh, int32_t cap_floats,
                       int32_t lmax, hipStream_t s) {
    SlabArgs a{};
    a.m = m;
    a.bw = bw;
    a.bh = bh;
    a.cap = cap_floats;
    a.lmax = lmax;
    a.m.groups_x = (m.cam.tile_w + bw - 1) / bw;
    int gy = (m.cam.tile_h + bh - 1) / bh;
    dim3 g((unsigned)(a.m.groups_x * gy)), b((unsigned)(bw * bh));
    size_t lds = (size_t)cap_floats * 4 + (mode == VR_COMPOSITE ? (size_t)m.lut.n * 16 : 0);
    switch (m.vol.dtype) {
        case VR_F32: return launch_slab_s<float>(a, mode, filter, g, b, lds, s);
        case VR_F16: return launch_slab_s<_Float16>(a, mode, filter, g, b, lds, s);
        default: return launch_slab_s<bf16_t>(a, mode, filter, g, b, lds, s);
    }
}

}  // namespace vr
