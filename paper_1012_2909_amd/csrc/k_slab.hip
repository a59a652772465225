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

// A 16-byte chunk of storage, already in registers -> floats in LDS.
template <typename S> __device__ __forceinline__ void put_raw(float *dst, uint4 v);
template <> __device__ __forceinline__ void put_raw<float>(float *dst, uint4 v) { *(uint4 *)dst = v; }
template <> __device__ __forceinline__ void put_raw<_Float16>(float *dst, uint4 v) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 a = __builtin_bit_cast(h2, v.x), b = __builtin_bit_cast(h2, v.y);
    const h2 c = __builtin_bit_cast(h2, v.z), d = __builtin_bit_cast(h2, v.w);
    *(float4 *)dst = make_float4((float)a[0], (float)a[1], (float)b[0], (float)b[1]);
    *(float4 *)(dst + 4) = make_float4((float)c[0], (float)c[1], (float)d[0], (float)d[1]);
}
template <> __device__ __forceinline__ void put_raw<bf16_t>(float *dst, uint4 v) {
    *(float4 *)dst = make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                                 __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
    *(float4 *)(dst + 4) = make_float4(__uint_as_float(v.z << 16), __uint_as_float(v.z & 0xffff0000u),
                                       __uint_as_float(v.w << 16), __uint_as_float(v.w & 0xffff0000u));
}

// Largest number of 16-byte chunks one thread stages per slab (all loads of
// a slab are in flight together; the slab thickness is chosen to fit).
constexpr int kMaxPasses = 16;

// Exact quotient of small non-negative integers, n <= 1024 and 1 <= d <=
// 1024, in FP32: (n + 1/2)/d lies at least 1/(2d) >= 2^-11 from any integer,
// while the rounding of the reciprocal (1 ulp) and of the product moves it by
// under n * 2^-22 <= 2^-12.
__device__ __forceinline__ int32_t sdiv(int32_t n, int32_t d) {
    return (int32_t)(((float)n + 0.5f) * __builtin_amdgcn_rcpf((float)d));
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
        // max(m, s) as the bare instruction: both are results of FP
        // arithmetic (or -inf), so the quieting the compiler would add for
        // fmaxf is not needed
        float r;
        asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(s), "v"(L.m));
        L.m = r;
        return true;
    }
    if (A.ckpt && (L.k & (kCkpt - 1)) == 0 && (L.k >> kCkptShift) < A.ckpt_segs) A.ckpt[(int64_t)(L.k >> kCkptShift) * npix + pix] = L.T;
    float4 c = lut_eval(lut, A.lut.n, A.lut.vmin, A.lut.scale, s);
    float ta = L.T * c.w;
    L.C0 = fmaf(ta, c.x, L.C0);
    L.C1 = fmaf(ta, c.y, L.C1);
    L.C2 = fmaf(ta, c.z, L.C2);
    L.T = L.use_log ? L.lt.step(c.w) : L.T - ta;
    return !(A.ert && L.T <= A.thr);
}

// Box of the slab [lo, lo + L) (corner index along W) in the copy's axis
// order: chunk-aligned origin fp0 along the fastest axis and the LDS
// dimensions; false if it is empty or too thin for the 2x2x2 footprint.
template <int W, int ORI, int EPC, int FILTER>
__device__ __forceinline__ bool slab_dims(const Frustum &F, int32_t lo, int32_t L, int32_t b0[3], int32_t &fp0,
                                          int32_t &Df, int32_t &Dm, int32_t &Ds) {
    constexpr int U = W == 0 ? 1 : 0, VV = W == 2 ? 1 : 2;
    constexpr int AF = ORI, AM = (ORI + 1) % 3, AS = (ORI + 2) % 3;
    int32_t lu, hu, lv, hv, lw, hw;
    slab_box(F, lo, L, lu, hu, lv, hv, lw, hw);
    int32_t b1[3];
    b0[W] = lw; b1[W] = hw; b0[U] = lu; b1[U] = hu; b0[VV] = lv; b1[VV] = hv;
    box_dims<EPC>(b0[AF], b1[AF], b0[AM], b1[AM], b0[AS], b1[AS], fp0, Df, Dm, Ds);
    if (Df <= 0 || Dm <= 0 || Ds <= 0) return false;
    return FILTER == VR_NEAREST || (Df >= 2 && Dm >= 2 && Ds >= 2);
}

// Samples of one lane inside the current slab, read from the LDS box.  The
// slab test and the end of the ray are one 64-bit comparison of the
// position along W with lim.  The box is in the copy's axis order: element
// strides 1, esm, ess for the fastest, middle and slowest axis (bM, bS in
// bytes), base the element offset of corner index (0,0,0); every box read is
// kept inside [0, maxoff] + the footprint.
template <int MODE, int FILTER, int W, int ORI, int SW>
__device__ __forceinline__ void lds_samples(LaneState &ls, const MarchArgs &A, const float4 *lut, int64_t pix,
                                            int64_t npix, const char *lds, int32_t esm, int32_t ess, int32_t base,
                                            uint32_t maxoff, uint32_t bM, uint32_t bS, int64_t lim) {
    int64_t q0 = ls.Q[0], q1 = ls.Q[1], q2 = ls.Q[2];
    const int64_t d0 = ls.D[0], d1 = ls.D[1], d2 = ls.D[2];
    int32_t k = ls.k;
    auto inside = [&](int64_t qw) { return SW > 0 ? qw < lim : qw >= lim; };
    if (inside(W == 0 ? q0 : (W == 1 ? q1 : q2))) do {
        // element offset: the fastest axis has stride 1, the other two go
        // through 24-bit multiplies; then bytes
        const int32_t i0 = fix_int(q0), i1 = fix_int(q1), i2 = fix_int(q2);
        const int32_t ia = ORI == 0 ? i0 : (ORI == 1 ? i1 : i2);
        const int32_t ib = ORI == 0 ? i1 : (ORI == 1 ? i2 : i0);
        const int32_t ic = ORI == 0 ? i2 : (ORI == 1 ? i0 : i1);
        const int32_t off = ia + __mul24(ib, esm) + __mul24(ic, ess) + base;
        VR_BOUNDS(A.vol, (uint32_t)off <= maxoff);   // the clamp below never engages
        const uint32_t o = min((uint32_t)off, maxoff) << 2;
        float s;
        if (FILTER == VR_NEAREST) {
            s = *(const float *)(lds + o);
        } else {
            const float fx = fix_frac(q0), fy = fix_frac(q1), fz = fix_frac(q2);
            // pairs along the fastest axis at the four (middle, slowest) corners
            const float *pa = (const float *)(lds + o), *pb = (const float *)(lds + o + bM);
            const float *pc = (const float *)(lds + o + bS), *pd = (const float *)(lds + o + bM + bS);
            const float a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
            const float c0 = pc[0], c1 = pc[1], e0 = pd[0], e1 = pd[1];
            float c000, c100, c010, c110, c001, c101, c011, c111;
            if (ORI == 0) {        // fastest x, then y, z
                c000 = a0; c100 = a1; c010 = b0; c110 = b1; c001 = c0; c101 = c1; c011 = e0; c111 = e1;
            } else if (ORI == 1) { // fastest y, then z, x
                c000 = a0; c010 = a1; c001 = b0; c011 = b1; c100 = c0; c110 = c1; c101 = e0; c111 = e1;
            } else {               // fastest z, then x, y
                c000 = a0; c001 = a1; c100 = b0; c101 = b1; c010 = c0; c011 = c1; c110 = e0; c111 = e1;
            }
            const float x00 = fmaf(fx, c100 - c000, c000), x10 = fmaf(fx, c110 - c010, c010);
            const float x01 = fmaf(fx, c101 - c001, c001), x11 = fmaf(fx, c111 - c011, c011);
            const float y0 = fmaf(fy, x10 - x00, x00), y1 = fmaf(fy, x11 - x01, x01);
            s = fmaf(fz, y1 - y0, y0);
        }
        q0 += d0; q1 += d1; q2 += d2;
        ls.k = k;
        const bool go = consume<MODE>(ls, A, lut, pix, npix, s);
        ++k;
        if (!go) { ls.stopped = true; break; }
    } while (inside(W == 0 ? q0 : (W == 1 ? q1 : q2)));
    ls.k = k;
    ls.Q[0] = q0; ls.Q[1] = q1; ls.Q[2] = q2;
}

// The same samples gathered straight from the volume (slabs whose box does
// not fit the LDS budget).
template <typename S, int MODE, int FILTER, int W, int SW>
__device__ __forceinline__ void gather_samples(LaneState &ls, const MarchArgs &A, const float4 *lut, int64_t pix,
                                               int64_t npix, int64_t lim) {
    for (;;) {
        const int64_t qw = ls.Q[W];
        if (SW > 0 ? !(qw < lim) : !(qw >= lim)) break;
        float fx = 0.f, fy = 0.f, fz = 0.f;
        if (FILTER == VR_TRILINEAR) { fx = fix_frac(ls.Q[0]); fy = fix_frac(ls.Q[1]); fz = fix_frac(ls.Q[2]); }
        const float s = gsample<S, FILTER>(A.vol, fix_int(ls.Q[0]), fix_int(ls.Q[1]), fix_int(ls.Q[2]), fx, fy, fz);
        ls.Q[0] += ls.D[0]; ls.Q[1] += ls.D[1]; ls.Q[2] += ls.D[2];
        const bool go = consume<MODE>(ls, A, lut, pix, npix, s);
        ++ls.k;
        if (!go) { ls.stopped = true; break; }
    }
}

// One slab of the march: corner indices [lo, lo + L) along W, and its voxel
// box (in the copy's axis order) if that is staged in LDS.
struct SlabPlan {
    int32_t lo, L, fp0, Df, Dm, Ds, b0[3];
    int32_t Pf;           // LDS row pitch (floats) of the box's fastest axis, >= Df
    bool lds;
};

// LDS row pitch for a box row of Df floats (a multiple of 4).
// (Padding the pitch to shift rows across LDS banks was measured: bank
// conflicts stayed within 4%, and the larger boxes slowed oblique views.)
__device__ __forceinline__ int32_t box_pitch(int32_t Df) { return Df; }

// The thickest slab starting at corner index cur (in the march direction),
// at most one thicker than the previous one and at most rem, whose box fits
// the LDS budget; a slab of thickness 1 that does not fit is marched with
// direct gathers.
template <typename S, int W, int ORI, int FILTER, int SW>
__device__ __forceinline__ SlabPlan plan_slab(const SlabArgs &SA, const Frustum &F, int32_t cur, int32_t Lprev,
                                              int32_t rem, int nthr) {
    constexpr int EPC = 16 / (int)sizeof(S);
    SlabPlan sl;
    auto fits = [&](int32_t Lt, SlabPlan &p) {
        p.lo = SW > 0 ? cur : cur - Lt + 1;
        p.L = Lt;
        p.lds = slab_dims<W, ORI, EPC, FILTER>(F, p.lo, Lt, p.b0, p.fp0, p.Df, p.Dm, p.Ds);
        p.Pf = box_pitch(p.Df);
        p.lds = p.lds && (int64_t)p.Pf * p.Dm * p.Ds <= SA.cap && p.Df / EPC <= nthr;
        return p.lds;
    };
    int32_t Lt = min(min(Lprev, SA.lmax), rem);
    if (fits(Lt, sl)) {
        // one thicker if the box has room for another plane
        const int64_t e = (int64_t)sl.Pf * sl.Dm * sl.Ds;
        SlabPlan g;
        if (Lt < min(SA.lmax, rem) && e + e / Lt <= SA.cap && fits(Lt + 1, g)) sl = g;
        return sl;
    }
    while (Lt > 1) {
        Lt = Lt > 8 ? Lt - (Lt >> 2) : Lt - 1;
        if (fits(Lt, sl)) break;
    }
    return sl;
}

// This thread's walk over the 16-byte chunks of a slab's box: rpp rows of
// cpr chunks per pass; thread t < rpp*cpr takes chunk t mod cpr of row
// t / cpr, then the same chunk rpp rows further on.  A round covers
// kMaxPasses passes.
template <typename S, int ORI>
struct BoxWalk {
    const S *gbase;
    float *dst;
    uint32_t goff, gA, gB;
    int32_t mm, mstep, Dm, rpp, rows, row0, dstep;
    bool on;

    __device__ __forceinline__ void init(const SlabPlan &sl, const VolDev &V, float *box, int tid, int nthr) {
        constexpr int AM = (ORI + 1) % 3, AS = (ORI + 2) % 3;
        constexpr int EPC = 16 / (int)sizeof(S);
        const uint32_t gstr[3] = {(uint32_t)V.sx, (uint32_t)V.sy, (uint32_t)V.sz};
        // cpr <= nthr <= 512 and rows per pass <= 512 (checked when the slab
        // was planned), so every quotient here is an exact sdiv
        const int32_t cpr = sl.Df / EPC;
        Dm = sl.Dm;
        rows = sl.Dm * sl.Ds;
        rpp = sdiv(nthr, cpr);
        row0 = sdiv(tid, cpr);
        const int32_t tx = tid - row0 * cpr;
        on = row0 < rpp;
        const int32_t Dq = min(Dm, 1024);                 // row0 < Dm whenever Dm > 1024
        const int32_t sq = sdiv(row0, Dq);
        mm = row0 - sq * Dq;
        const int32_t sstep = sdiv(rpp, Dq);
        mstep = rpp - sstep * Dq;
        gbase = (const S *)V.data + ((size_t)(sl.b0[AS] + 1) * gstr[AS] + (size_t)(sl.b0[AM] + 1) * gstr[AM] +
                                     (size_t)sl.fp0);
        goff = (uint32_t)sq * gstr[AS] + (uint32_t)mm * gstr[AM] + (uint32_t)(tx * EPC);
        gA = (uint32_t)sstep * gstr[AS] + (uint32_t)mstep * gstr[AM];
        gB = gstr[AS] - (uint32_t)Dm * gstr[AM];
        dst = box + (row0 * sl.Pf + tx * EPC);
        dstep = rpp * sl.Pf;
    }
    // Issue the loads of the round whose first row is r0; nothing waits.
    // Loads and stores are unconditional (a chunk past the box reloads the
    // box's first chunk and is stored to the spare slot after the box), so
    // that no branch splits the sequence and all loads stay in flight.
    __device__ __forceinline__ void load(uint4 (&raw)[kMaxPasses], int32_t r0) {
#pragma unroll
        for (int p = 0; p < kMaxPasses; ++p) {
            const bool ok = on && r0 + p * rpp < rows;
            raw[p] = *(const uint4 *)(gbase + (ok ? goff : 0u));
            goff += gA;
            mm += mstep;
            if (mm >= Dm) { mm -= Dm; goff += gB; }
        }
    }
    __device__ __forceinline__ void store(const uint4 (&raw)[kMaxPasses], int32_t r0, float *spare) {
#pragma unroll
        for (int p = 0; p < kMaxPasses; ++p) {
            const bool ok = on && r0 + p * rpp < rows;
            put_raw<S>(ok ? dst : spare, raw[p]);
            dst += dstep;
        }
    }
};

// The slab march for slab axis W (0, 1, 2 = x, y, z) and direction SW over
// the copy whose fastest axis is ORI.  The slabs cover the corner-index range
// [wlo, whi] of the bundle's regular lanes in order; each slab is as thick
// as the LDS budget allows at that depth (a perspective bundle widens with
// distance), at most lmax.  The box loads of the next slab are issued before
// the current slab is sampled, so their latency hides behind the sampling.
// The plan of a slab is the same for every lane, so the first wave alone
// computes it, one slab ahead, into two LDS slots (plans, reused from the
// corner-ray scratch): slab i + 2 is planned while slab i is sampled, into the
// slot of slab i, which every thread read before that iteration's first
// barrier; the barriers of iteration i + 1 order the write before the reads.
template <typename S, int MODE, int FILTER, int W, int ORI, int SW>
__device__ __forceinline__ void run_slabs(const SlabArgs &SA, const Frustum &F, LaneState &ls, bool active,
                                          int32_t wlo, int32_t whi, float *box, const float4 *lut, int64_t pix,
                                          int64_t npix, SlabPlan *plans) {
    const MarchArgs &A = SA.m;
    const VolDev &V = A.vol;
    constexpr int AM = (ORI + 1) % 3, AS = (ORI + 2) % 3;   // middle and slowest axis
    const int tid = threadIdx.x, nthr = blockDim.x;
    const bool planner = tid < 64;
    // the position along W of the lane's last sample
    const int64_t qlast = ls.Q[W] + (int64_t)(ls.n > 0 ? ls.n - 1 : 0) * ls.D[W];
    auto remaining = [&](int32_t c) { return SW > 0 ? whi - c + 1 : c - wlo + 1; };
    auto advance = [&](int32_t c, int32_t L) { return SW > 0 ? c + L : c - L; };
    // the plan of the slab after the one starting at c with thickness L (none past the range)
    auto plan_after = [&](int32_t c, int32_t L) {
        SlabPlan p{};
        const int32_t cn = advance(c, L);
        if (remaining(cn) > 0) p = plan_slab<S, W, ORI, FILTER, SW>(SA, F, cn, L, remaining(cn), nthr);
        return p;
    };
    int32_t cur = SW > 0 ? wlo : whi;                 // first corner index not yet covered
    __syncthreads();                                  // the plan slots may still hold the corner rays
    if (planner) {
        const SlabPlan p0 = plan_slab<S, W, ORI, FILTER, SW>(SA, F, cur, SA.lmax, remaining(cur), nthr);
        const SlabPlan p1 = plan_after(cur, p0.L);
        if (tid == 0) {
            plans[0] = p0;
            plans[1] = p1;
        }
    }
    __syncthreads();
    uint4 raw[kMaxPasses];
    BoxWalk<S, ORI> wk;
    SlabPlan nxt = plans[0];
    if (nxt.lds) {
        wk.init(nxt, V, box, tid, nthr);
        wk.load(raw, wk.row0);
    }
    int32_t slot = 1;                                 // slot of the next slab's plan
    while (__syncthreads_or(active)) {
        if (remaining(cur) <= 0) break;
        const SlabPlan sl = nxt;
        if (sl.lds) {
            float *spare = box + SA.cap;                  // 8 floats past the largest box
            wk.store(raw, wk.row0, spare);
            for (int32_t r0 = wk.row0 + wk.rpp * kMaxPasses; r0 < wk.rows; r0 += wk.rpp * kMaxPasses) {
                wk.load(raw, r0);
                wk.store(raw, r0, spare);
            }
            __syncthreads();
        }
        // the next slab's plan from its slot, and its loads; the first wave
        // plans the slab after it into the other slot
        cur = advance(cur, sl.L);
        if (remaining(cur) > 0) {
            nxt = plans[slot];
            if (nxt.lds) {
                wk.init(nxt, V, box, tid, nthr);
                wk.load(raw, wk.row0);
            }
            slot ^= 1;
            if (planner) {
                const SlabPlan p2 = plan_after(cur, nxt.L);
                if (tid == 0) plans[slot] = p2;
            }
        }
        if (active) {
            const int64_t wedge = (int64_t)(SW > 0 ? sl.lo + sl.L : sl.lo) * 4294967296LL;   // in 32.32
            const int64_t lim = SW > 0 ? min(wedge, qlast + 1) : max(wedge, qlast);
            if (sl.lds) {
                // element strides of the box (fastest axis 1) and the offset of
                // corner index (0,0,0)
                const int32_t esm = sl.Pf, ess = sl.Pf * sl.Dm;
                const int32_t base = -((sl.fp0 - 1) + sl.b0[AM] * esm + sl.b0[AS] * ess);
                const int32_t foot = FILTER == VR_TRILINEAR ? esm + ess + 1 : 0;
                const uint32_t maxoff = (uint32_t)(sl.Pf * sl.Dm * sl.Ds - 1 - foot);
                lds_samples<MODE, FILTER, W, ORI, SW>(ls, A, lut, pix, npix, (const char *)box, esm, ess, base,
                                                      maxoff, (uint32_t)(4 * esm), (uint32_t)(4 * ess), lim);
            } else {
                gather_samples<S, MODE, FILTER, W, SW>(ls, A, lut, pix, npix, lim);
            }
            if (ls.stopped || ls.k >= ls.n) active = false;
        }
    }
}

// The lanes whose pixel (px, py) is a corner of the bundle [bx0, cx1] x
// [by0, cy1] store their ray (origin minus (sx, sy, sz), direction); then a
// barrier.  A lane may hold several corners of a one-pixel-wide bundle.
__device__ __forceinline__ void publish_corners(double *corners, int px, int py, int bx0, int by0, int cx1, int cy1,
                                                const Ray &r, double sx, double sy, double sz) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (px == ((c & 1) ? cx1 : bx0) && py == ((c & 2) ? cy1 : by0)) {
            double *q = corners + 6 * c;
            q[0] = r.ox - sx; q[1] = r.oy - sy; q[2] = r.oz - sz;
            q[3] = r.dx; q[4] = r.dy; q[5] = r.dz;
        }
    __syncthreads();
}

__device__ __forceinline__ void read_corners(const double *corners, double (&ox)[4], double (&oy)[4],
                                             double (&oz)[4], double (&dx)[4], double (&dy)[4], double (&dz)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double *q = corners + 6 * c;
        ox[c] = q[0]; oy[c] = q[1]; oz[c] = q[2];
        dx[c] = q[3]; dy[c] = q[4]; dz[c] = q[5];
    }
}

// One bundle of bw x bh pixels whose top-left pixel is (bx0, by0) of the
// viewport in SA.m (called by every thread of the workgroup).  smem holds the
// table (composite) followed by the voxel box; red is a 16-int scratch and
// corners a 24-double one.
template <typename S, int MODE, int FILTER, int ORI>
__device__ __forceinline__ void slab_bundle(const SlabArgs &SA, int bx0, int by0, float *smem, int32_t *red,
                                            double *corners) {
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
    // the corner rays are the rays of the lanes at the bundle's corner pixels
    // (all inside the viewport), shared through LDS
    publish_corners(corners, px, py, bx0, by0, cx1, cy1, r, 0.0, 0.0, 0.0);
    double cox[4], coy[4], coz[4], cdx[4], cdy[4], cdz[4];
    read_corners(corners, cox, coy, coz, cdx, cdy, cdz);
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
    if (MODE == VR_COMPOSITE) {   // table to LDS (after the FP64 set-up)
        for (int i = tid; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
        __syncthreads();
    }
    const int64_t npix = (int64_t)A.cam.tile_w * A.cam.tile_h;
    const int64_t pix = (int64_t)py * A.cam.tile_w + px;

    if (wlo <= whi && bundle_ok) {
        const bool active = reg;
        SlabPlan *plans = (SlabPlan *)corners;        // the corner rays have been read
        static_assert(2 * sizeof(SlabPlan) <= 24 * sizeof(double), "two slab plans fit the corner-ray scratch");
        if (sw > 0) {
            if (w == 0) run_slabs<S, MODE, FILTER, 0, ORI, 1>(SA, F, ls, active, wlo, whi, box, lut, pix, npix, plans);
            else if (w == 1) run_slabs<S, MODE, FILTER, 1, ORI, 1>(SA, F, ls, active, wlo, whi, box, lut, pix, npix, plans);
            else run_slabs<S, MODE, FILTER, 2, ORI, 1>(SA, F, ls, active, wlo, whi, box, lut, pix, npix, plans);
        } else {
            if (w == 0) run_slabs<S, MODE, FILTER, 0, ORI, -1>(SA, F, ls, active, wlo, whi, box, lut, pix, npix, plans);
            else if (w == 1) run_slabs<S, MODE, FILTER, 1, ORI, -1>(SA, F, ls, active, wlo, whi, box, lut, pix, npix, plans);
            else run_slabs<S, MODE, FILTER, 2, ORI, -1>(SA, F, ls, active, wlo, whi, box, lut, pix, npix, plans);
        }
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
__global__ __launch_bounds__(512) void k_slab(SlabArgs SA) {
    extern __shared__ float smem[];
    __shared__ int32_t red[16];
    __shared__ double corners[24];
    int32_t gbx, gby;
    tile_xy(blockIdx.x, gridDim.x, SA.m.groups_x, (int32_t)(gridDim.x / (uint32_t)SA.m.groups_x), SA.m.order,
            SA.m.tile_perm, gbx, gby);
    slab_bundle<S, MODE, FILTER, ORI>(SA, gbx * SA.bw, gby * SA.bh, smem, red, corners);
}

// K3 with LDS-staged voxel boxes: one workgroup renders a 16 x 16 tile of one
// brick's footprint (the same job table as k_brick).  Each lane's ray is set
// up on the whole cube, and the run of its global samples whose positions
// lie in the brick (exact fixed-point membership, half-open boxes) is then
// marched in the brick's own block, as a one-brick volume whose origin is the
// brick's corner: the slab machinery of the bundle kernel stages the boxes
// of that block in LDS.  The arithmetic is that of k_brick (same positions,
// same interpolation and table, the brick's own early stop), so both give
// the same partials.
template <typename S, int MODE, int FILTER>
__global__ __launch_bounds__(256) void k_brick_slab(SlabArgs SA, const BrickJob *__restrict__ jobs, int32_t n_jobs) {
    extern __shared__ float smem[];
    __shared__ int32_t red[16];
    __shared__ double corners[24];
    const int32_t t = blockIdx.x;
    int32_t lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const BrickJob J = jobs[lo];
    const MarchArgs &A = SA.m;
    const VolDev &Vc = A.vol;                            // the whole bricked cube
    const int tid = threadIdx.x;
    const int32_t tl = t - J.tile_begin;
    const int32_t bx0 = (tl % J.tiles_x) * 16, by0 = (tl / J.tiles_x) * 16;
    const int32_t lx = bx0 + (tid & 15), ly = by0 + (tid >> 4);
    const bool valid = lx < J.w && ly < J.h;
    const int px = J.x0 + lx, py = J.y0 + ly;
    float4 *lut = (float4 *)smem;
    float *box = smem + (MODE == VR_COMPOSITE ? 4 * A.lut.n : 0);

    // the brick as a one-brick volume: local voxel (-1,-1,-1) is element 0
    const int32_t og[3] = {J.bx * Vc.Bx, J.by * Vc.By, J.bz * Vc.Bz};
    SlabArgs S2 = SA;
    VolDev &V = S2.m.vol;
    V.data = J.brick ? J.brick
                     : (const void *)((const S *)Vc.data +
                                      ((int64_t)(J.bz * Vc.nby + J.by) * Vc.nbx + J.bx) * Vc.brick_elems);
    V.nx = Vc.Bx; V.ny = Vc.By; V.nz = Vc.Bz;
    V.sx = 1; V.sy = Vc.Px; V.sz = Vc.Px * Vc.Py;
    V.ori = 0; V.single = 1; V.orients = 1;

    Ray r{};
    if (valid) make_ray(A.cam, Vc, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    int64_t P[3], D[3];
    fix_start(r, A.step, 0, 0.0, P, D);
    int64_t k0 = 0, k1 = r.n;
    {
        const int64_t one = (int64_t)1 << 32;
        const int32_t bh[3] = {min(og[0] + Vc.Bx, Vc.nx), min(og[1] + Vc.By, Vc.ny), min(og[2] + Vc.Bz, Vc.nz)};
        const int32_t N[3] = {Vc.nx, Vc.ny, Vc.nz};
        if (k1 > 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                int64_t a0 = k0, a1 = k1;
                const int64_t lo_f = og[a] == 0 ? INT64_MIN / 4 : (int64_t)og[a] * one;
                const int64_t hi_f = bh[a] == N[a] ? INT64_MAX / 4 : (int64_t)bh[a] * one;
                brick_axis_range(P[a], D[a], lo_f, hi_f, a0, a1);
                k0 = max(k0, a0);
                k1 = min(k1, a1);
            }
        }
    }
    const int64_t sh = FILTER == VR_TRILINEAR ? ((int64_t)1 << 31) : 0;   // corner grid q = p - 1/2
    LaneState ls;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ls.Q[a] = P[a] - sh + k0 * D[a] - (int64_t)og[a] * ((int64_t)1 << 32);
        ls.D[a] = D[a];
    }
    ls.n = (int32_t)max(k1 - k0, (int64_t)0);
    ls.k = 0;
    ls.m = -INFINITY;
    ls.T = 1.0f;
    ls.C0 = ls.C1 = ls.C2 = 0.0f;
    ls.use_log = false;                                  // the brick partial keeps the product, as k_brick does
    ls.stopped = false;

    // the bundle's slab axis and corner rays, in brick-local coordinates
    const int cx1 = min(bx0 + 16, J.w) - 1, cy1 = min(by0 + 16, J.h) - 1;
    // the corner rays (in brick-local coordinates) are the rays of the lanes at
    // the tile's corner pixels, shared through LDS
    publish_corners(corners, lx, ly, bx0, by0, cx1, cy1, r, (double)og[0], (double)og[1], (double)og[2]);
    double cox[4], coy[4], coz[4], cdx[4], cdy[4], cdz[4];
    read_corners(corners, cox, coy, coz, cdx, cdy, cdz);
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
    F.h = FILTER == VR_TRILINEAR ? 0.5f : 0.0f;
    const int64_t Qw0 = w == 0 ? ls.Q[0] : (w == 1 ? ls.Q[1] : ls.Q[2]);
    const int64_t Dw = w == 0 ? ls.D[0] : (w == 1 ? ls.D[1] : ls.D[2]);
    const double rdw = w == 0 ? r.dx : (w == 1 ? r.dy : r.dz);
    const bool reg = valid && ls.n > 0 && bundle_ok && (Dw > 0) == (sw > 0) && fabs(rdw) >= 0.2;
    int32_t wlo, whi;
    {
        const int32_t first = fix_int(Qw0), last = fix_int(Qw0 + (int64_t)(ls.n > 0 ? ls.n - 1 : 0) * Dw);
        int32_t a = reg ? min(first, last) : INT32_MAX, b = reg ? max(first, last) : INT32_MIN;
        wg_minmax(a, b, red);
        wlo = a;
        whi = b;
    }
    if (MODE == VR_COMPOSITE) {
        for (int i = tid; i < A.lut.n; i += blockDim.x) lut[i] = A.lut.rgba[i];
        __syncthreads();
    }
    if (wlo <= whi && bundle_ok) {
        if (sw > 0) {
            if (w == 0) run_slabs<S, MODE, FILTER, 0, 0, 1>(S2, F, ls, reg, wlo, whi, box, lut, 0, 0, (SlabPlan *)corners);
            else if (w == 1) run_slabs<S, MODE, FILTER, 1, 0, 1>(S2, F, ls, reg, wlo, whi, box, lut, 0, 0, (SlabPlan *)corners);
            else run_slabs<S, MODE, FILTER, 2, 0, 1>(S2, F, ls, reg, wlo, whi, box, lut, 0, 0, (SlabPlan *)corners);
        } else {
            if (w == 0) run_slabs<S, MODE, FILTER, 0, 0, -1>(S2, F, ls, reg, wlo, whi, box, lut, 0, 0, (SlabPlan *)corners);
            else if (w == 1) run_slabs<S, MODE, FILTER, 1, 0, -1>(S2, F, ls, reg, wlo, whi, box, lut, 0, 0, (SlabPlan *)corners);
            else run_slabs<S, MODE, FILTER, 2, 0, -1>(S2, F, ls, reg, wlo, whi, box, lut, 0, 0, (SlabPlan *)corners);
        }
    }
    // lanes outside the slab scheme (and any samples left over): direct gathers
    if (valid && !ls.stopped && ls.k < ls.n) {
        while (ls.k < ls.n) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
            if (FILTER == VR_TRILINEAR) { fx = fix_frac(ls.Q[0]); fy = fix_frac(ls.Q[1]); fz = fix_frac(ls.Q[2]); }
            const float s = gsample<S, FILTER>(V, fix_int(ls.Q[0]), fix_int(ls.Q[1]), fix_int(ls.Q[2]), fx, fy, fz);
            ls.Q[0] += ls.D[0]; ls.Q[1] += ls.D[1]; ls.Q[2] += ls.D[2];
            const bool go = consume<MODE>(ls, S2.m, lut, 0, 0, s);
            ++ls.k;
            if (!go) break;
        }
    }
    if (valid) {
        const int64_t o = (int64_t)ly * J.w + lx;
        if (MODE == VR_MIP) J.data[o] = ls.m;
        else ((float4 *)J.data)[o] = make_float4(ls.C0, ls.C1, ls.C2, 1.0f - ls.T);
    }
}

// K6: persistent workgroups pull bundles from an atomic queue until every
// bundle of every view is done (each workgroup exits once the counter passes
// the item count).  Items are numbered view by view, largest views first.
template <typename S, int MODE, int FILTER>
__global__ __launch_bounds__(512) void k_batch(BatchArgs B) {
    extern __shared__ float smem[];
    __shared__ int32_t red[16];
    __shared__ double corners[24];
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
        SA.m.vol.data = V.vdata;
        SA.m.vol.sx = V.vsx;
        SA.m.vol.sy = V.vsy;
        SA.m.vol.sz = V.vsz;
        SA.m.vol.ori = V.ori;
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
        if (V.ori == 1) slab_bundle<S, MODE, FILTER, 1>(SA, bx0, by0, smem, red, corners);
        else if (V.ori == 2) slab_bundle<S, MODE, FILTER, 2>(SA, bx0, by0, smem, red, corners);
        else slab_bundle<S, MODE, FILTER, 0>(SA, bx0, by0, smem, red, corners);
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
    const size_t lds = (size_t)a.cap * 4 + 32 + (MODE == VR_COMPOSITE ? (size_t)a.lut_n * 16 : 0);
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


template <typename S, int MODE, int FILTER>
static hipError_t launch_brick_slab_t(const SlabArgs &a, const BrickJob *jobs, int32_t n, int32_t tiles, size_t lds,
                                      hipStream_t s) {
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_brick_slab<S, MODE, FILTER>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_brick_slab<S, MODE, FILTER>), dim3((unsigned)tiles), dim3(256), lds, s, a, jobs, n);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_brick_slab_s(const SlabArgs &a, int32_t mode, int32_t filter, const BrickJob *jobs,
                                      int32_t n, int32_t tiles, size_t lds, hipStream_t s) {
    if (mode == VR_MIP) {
        if (filter == VR_NEAREST) return launch_brick_slab_t<S, VR_MIP, VR_NEAREST>(a, jobs, n, tiles, lds, s);
        return launch_brick_slab_t<S, VR_MIP, VR_TRILINEAR>(a, jobs, n, tiles, lds, s);
    }
    if (filter == VR_NEAREST) return launch_brick_slab_t<S, VR_COMPOSITE, VR_NEAREST>(a, jobs, n, tiles, lds, s);
    return launch_brick_slab_t<S, VR_COMPOSITE, VR_TRILINEAR>(a, jobs, n, tiles, lds, s);
}

hipError_t launch_bricks_slab(const MarchArgs &m, int32_t mode, int32_t filter, const BrickJob *jobs_dev,
                              int32_t n_jobs, int32_t total_tiles, int32_t cap_floats, int32_t lmax, hipStream_t s) {
    if (n_jobs <= 0 || total_tiles <= 0) return hipSuccess;
    SlabArgs a{};
    a.m = m;
    a.bw = a.bh = 16;
    const int32_t avail = (160 * 1024 - 1024 - 32 - (mode == VR_COMPOSITE ? m.lut.n * 16 : 0)) / 4;
    a.cap = cap_floats < avail ? cap_floats : avail;
    a.lmax = lmax;
    const size_t lds = (size_t)a.cap * 4 + 32 + (mode == VR_COMPOSITE ? (size_t)m.lut.n * 16 : 0);
    switch (m.vol.dtype) {
        case VR_F32: return launch_brick_slab_s<float>(a, mode, filter, jobs_dev, n_jobs, total_tiles, lds, s);
        case VR_F16: return launch_brick_slab_s<_Float16>(a, mode, filter, jobs_dev, n_jobs, total_tiles, lds, s);
        default: return launch_brick_slab_s<bf16_t>(a, mode, filter, jobs_dev, n_jobs, total_tiles, lds, s);
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

// ---- costliest bundles first --------------------------------------------
// A CU starts the next workgroup when one finishes, in id order, so the frame
// ends when the last-started bundles end.  Bundles differ in cost by up to
// ~7x within one view (rays at 45 degrees between two axes make the widest
// boxes), and a heavy one that starts late stretches the frame.  The bundles
// are therefore launched in decreasing order of an estimate of the 128-byte
// lines their boxes fetch: the boxes of two slabs 8 corner indices thick, at
// a quarter and three quarters of the depth range the bundle's corner and
// centre rays span along their dominant axis, each row counted at the mean
// number of lines a row of its bytes touches from a random 4-byte offset,
// times the range over 8.  The estimate orders the tiles only: every bundle
// renders the same pixels in any order.

// Estimated lines of the bundle with corner pixels (x0, y0), (x1, y1).
__device__ double bundle_lines(const MarchArgs &A, int32_t x0, int32_t y0, int32_t x1, int32_t y1) {
    const CamDev &c = A.cam;
    const VolDev &v = A.vol;
    const double N[3] = {(double)v.nx, (double)v.ny, (double)v.nz};
    double o[4][3], d[4][3], dc[3] = {0.0, 0.0, 0.0};
    double te[5], tx[5], ow[5][3], dw[5][3];
    bool hit = false;
    for (int k = 0; k < 5; ++k) {
        const int32_t px = k < 4 ? ((k & 1) ? x1 : x0) : (x0 + x1) / 2;
        const int32_t py = k < 4 ? ((k & 2) ? y1 : y0) : (y0 + y1) / 2;
        Ray r{};
        make_ray(c, v, c.tile_x0 + px, c.tile_y0 + py, A.step, r);
        ow[k][0] = r.ox; ow[k][1] = r.oy; ow[k][2] = r.oz;
        dw[k][0] = r.dx; dw[k][1] = r.dy; dw[k][2] = r.dz;
        te[k] = r.t0;
        tx[k] = r.n > 0 ? r.t1 : -1.0;
        hit = hit || r.n > 0;
        if (k < 4)
            for (int a = 0; a < 3; ++a) { o[k][a] = ow[k][a]; d[k][a] = dw[k][a]; dc[a] += dw[k][a]; }
    }
    if (!hit) return 0.0;
    int w = 0;
    if (fabs(dc[1]) > fabs(dc[w])) w = 1;
    if (fabs(dc[2]) > fabs(dc[w])) w = 2;
    double lo = 1e300, hi = -1e300;
    for (int k = 0; k < 5; ++k) {
        if (tx[k] < 0.0) continue;
        const double pa = ow[k][w] + te[k] * dw[k][w], pb = ow[k][w] + tx[k] * dw[k][w];
        lo = fmin(lo, fmin(pa, pb));
        hi = fmax(hi, fmax(pa, pb));
    }
    const int f = v.ori, m = (v.ori + 1) % 3, sl = (v.ori + 2) % 3;
    const double es = v.dtype == VR_F32 ? 4.0 : 2.0;
    double lines = 0.0;
    for (int e = 0; e < 2; ++e) {
        const double p0 = lo + (hi - lo) * (0.25 + 0.5 * e) - 4.0, p1 = p0 + 8.0;
        double ext[3];
        for (int a = 0; a < 3; ++a) {
            if (a == w) { ext[a] = 9.0; continue; }
            double mn = 1e300, mx = -1e300;
            for (int k = 0; k < 4; ++k) {
                // rays shallower than 0.2 along w are gathered directly by the
                // bundle kernel; the clamp keeps their estimate finite and large
                const double dwk = fabs(d[k][w]) < 0.2 ? copysign(0.2, d[k][w]) : d[k][w];
                for (int q = 0; q < 2; ++q) {
                    const double pw = q ? p1 : p0;
                    const double x = o[k][a] + (pw - o[k][w]) / dwk * d[k][a];
                    mn = fmin(mn, x);
                    mx = fmax(mx, x);
                }
            }
            ext[a] = fmin(fmax(floor(mx) - floor(mn) + 2.0, 2.0), N[a] + 2.0);
        }
        lines += ext[m] * ext[sl] * (floor((ext[f] * es + 124.0) / 128.0) + 1.0);
    }
    return lines * 0.5 * (hi - lo + 1.0) / 8.0;
}

// The estimate of every tile as a sort key: its logarithm in buckets 2^(1/8)
// apart, costliest first (key 0).
__global__ __launch_bounds__(256) void k_tile_cost(MarchArgs A, int32_t bw, int32_t bh, int32_t ntiles,
                                                    uint8_t *key) {
    const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= ntiles) return;
    const int32_t tx = t % A.groups_x, ty = t / A.groups_x;
    const int32_t x0 = tx * bw, y0 = ty * bh;
    const int32_t x1 = min(x0 + bw, A.cam.tile_w) - 1, y1 = min(y0 + bh, A.cam.tile_h) - 1;
    const double lines = bundle_lines(A, x0, y0, x1, y1);
    key[t] = (uint8_t)(255 - (int32_t)fmin(log2(lines + 1.0) * 8.0, 255.0));
}

// One workgroup: a counting sort of the tiles by key in LDS, written as the
// permutation (the order within a key is arbitrary).
__global__ __launch_bounds__(1024) void k_tile_sort(int32_t ntiles, const uint8_t *key, int32_t *perm) {
    __shared__ int32_t hist[256];
    const int tid = threadIdx.x;
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    for (int32_t t = tid; t < ntiles; t += 1024) atomicAdd(&hist[key[t]], 1);
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int i = 0; i < 256; ++i) {
            const int32_t h = hist[i];
            hist[i] = run;
            run += h;
        }
    }
    __syncthreads();
    for (int32_t t = tid; t < ntiles; t += 1024) perm[atomicAdd(&hist[key[t]], 1)] = t;
}

int64_t slab_order_bytes(int32_t w, int32_t h, int32_t bw, int32_t bh) {
    const int64_t n = (int64_t)((w + bw - 1) / bw) * ((h + bh - 1) / bh);
    return (n * 4 + 255) / 256 * 256 + n;
}

hipError_t launch_slab(const MarchArgs &m, int32_t mode, int32_t filter, int32_t bw, int32_t bh, int32_t cap_floats,
                       int32_t lmax, hipStream_t s) {
    SlabArgs a{};
    a.m = m;
    a.bw = bw;
    a.bh = bh;
    // dynamic LDS = box + spare slot + table must fit next to the kernel's
    // static LDS (under 1 KiB) in the 160 KiB of a CU
    const int32_t avail = (160 * 1024 - 1024 - 32 - (mode == VR_COMPOSITE ? m.lut.n * 16 : 0)) / 4;
    a.cap = cap_floats < avail ? cap_floats : avail;
    a.lmax = lmax;
    a.m.groups_x = (m.cam.tile_w + bw - 1) / bw;
    int gy = (m.cam.tile_h + bh - 1) / bh;
    dim3 g((unsigned)(a.m.groups_x * gy)), b((unsigned)(bw * bh));
    if (a.m.order == 3 && a.m.tile_perm && a.m.tile_key) {
        const int32_t n = a.m.groups_x * gy;
        hipLaunchKernelGGL(k_tile_cost, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.m, bw, bh, n,
                           a.m.tile_key);
        hipLaunchKernelGGL(k_tile_sort, dim3(1), dim3(1024), 0, s, n, (const uint8_t *)a.m.tile_key, a.m.tile_perm);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    } else {
        a.m.tile_perm = nullptr;
    }
    // box budget + one spare 8-float slot + the table (composite)
    size_t lds = (size_t)a.cap * 4 + 32 + (mode == VR_COMPOSITE ? (size_t)m.lut.n * 16 : 0);
    switch (m.vol.dtype) {
        case VR_F32: return launch_slab_s<float>(a, mode, filter, g, b, lds, s);
        case VR_F16: return launch_slab_s<_Float16>(a, mode, filter, g, b, lds, s);
        default: return launch_slab_s<bf16_t>(a, mode, filter, g, b, lds, s);
    }
}

}  // namespace vr
