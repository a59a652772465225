// k_mipblk.hip -- K8: maximum-intensity projection in object order.
//
// The maximum of a ray's samples does not depend on the order they are
// taken in, so a MIP frame can be computed block by block of the volume
// instead of ray by ray: every voxel is then read from HBM about once per
// frame, where a bundle of rays marching in depth reads the voxel boxes of
// its own frustum (boxes of neighbouring bundles overlap, and their rows
// start and end inside cache lines).
//
// The corner-index space [-1, N] of each axis (the integer part of a
// sample's fixed-point position, see fix_start) is partitioned into blocks of
// SX x SY x SZ; block j of an axis holds corner indices [j*S - 1, j*S + S - 2].
// Every sample lies in exactly one block.  A workgroup walks a run of blocks
// along x; for each block it
//   - copies the block's voxels (its corner indices and the +1 neighbours,
//     (SX+1) x (SY+1) x (SZ+1)) into LDS: from the line copy of an FP32
//     three-copy layout (SX = 31, one whole 128-byte line per row), else from
//     the padded x-fastest copy (SX = 32: rows of 33 elements, which start and
//     end inside lines);
//   - bounds the block's pixels by projecting the corners of the part of the
//     cube its samples can occupy (the hull's bounding rectangle with a small
//     margin; the whole tile when the region comes within a voxel of the
//     eye's plane);
//   - gives each lane one pixel of the rectangle: from the pixel's ray record
//     (fixed-point start, step and sample count, computed once per frame) the
//     lane finds the run [kb, ke) of samples inside the block -- a float
//     estimate widened by two samples, then trimmed with exact integer
//     comparisons, so the run is exact -- takes the maximum of those samples
//     from LDS and merges it into the pixel with one atomic maximum.
// Samples are interpolated with the same arithmetic as the marching kernels
// (same positions, same fused multiply-adds), and a maximum is exact, so the
// image equals theirs bit for bit.  The atomic maximum works on an
// order-preserving unsigned encoding of the float; the frame starts at the
// encoding of -inf (a miss) and is decoded in place at the end.
#include "vr_internal.h"

namespace vr {

// Ray of one tile pixel, in the fixed point of the marching kernels.
struct RayRec {
    int64_t Q[3];         // position of sample 0 minus the corner-grid shift, 32.32
    int64_t D[3];         // increment per sample, 32.32
    int32_t n;            // samples
    float rd[3];          // 1/D (in samples per 32.32 unit), for the run estimate
};
static_assert(sizeof(RayRec) == 64, "ray record is one 64-byte line");

constexpr int kBX = 32;                          // block edge along x (corner indices) on the x-fastest copy
constexpr int kBXL = 31;                         // block edge along x on the line copy: one line per row
constexpr int kPX = 36;                          // LDS row pitch (floats): kBX + 1 rounded up to 4
constexpr int kMaxRun = 64;                      // blocks along x per workgroup

// Waves per SIMD that the kernel's registers are budgeted for.  A CU has
// four SIMDs and 160 KiB of LDS; a 256-thread workgroup puts one wave on each
// SIMD, so the budget matches the number of workgroups the LDS of a block of
// BY x BZ rows leaves room for (the voxel box, its spare slot and the run's
// rectangles; at most 4), and registers do not cut the occupancy below what
// the LDS allows.  Other workgroup sizes keep two waves per SIMD (the FP32
// staging of a 512-thread group does not fit the 128 registers of four).
template <int BY, int BZ, int NT> constexpr int waves_per_simd() {
    constexpr int bytes = 4 * (kPX * (BY + 1) * (BZ + 1) + 8) + kMaxRun * 16;
    return NT != 256 ? 2 : (163840 / bytes < 4 ? 163840 / bytes : 4);
}

// Order-preserving map of a (non-NaN) float onto uint32 and back.
__device__ __forceinline__ uint32_t mip_enc(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float mip_dec(uint32_t e) {
    return __uint_as_float((e & 0x80000000u) ? (e & 0x7fffffffu) : ~e);
}

// Ray records of every tile pixel, and the frame set to the encoding of -inf.
template <int FILTER>
__global__ __launch_bounds__(256) void k_raytable(MarchArgs A, RayRec *tab) {
    const int64_t npix = (int64_t)A.cam.tile_w * A.cam.tile_h;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const int px = (int)(i % A.cam.tile_w), py = (int)(i / A.cam.tile_w);
    Ray r{};
    make_ray(A.cam, A.vol, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
    RayRec rec;
    fix_start(r, A.step, 0, FILTER == VR_TRILINEAR ? 0.5 : 0.0, rec.Q, rec.D);
    rec.n = r.n;
#pragma unroll
    for (int a = 0; a < 3; ++a) rec.rd[a] = rec.D[a] != 0 ? (float)(1.0 / (double)rec.D[a]) : 0.0f;
    tab[i] = rec;
    ((uint32_t *)A.out)[i] = mip_enc(-INFINITY);
}

__global__ __launch_bounds__(256) void k_mip_decode(uint32_t *out, int64_t npix) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npix) ((float *)out)[i] = mip_dec(out[i]);
}

struct BlockArgs {
    MarchArgs m;          // vol: the x-fastest copy
    const RayRec *tab;
    int32_t nb[3];        // blocks per axis
    int32_t run;          // blocks along x per workgroup
    int32_t runs_x;       // runs per row of blocks
};

// Projected pixel rectangle (tile-local, half-open) of the sample region of
// corner-index box [lo, hi]; empty when it misses the tile.
__device__ __forceinline__ void block_rect(const CamDev &c, const VolDev &v, const int32_t lo[3],
                                           const int32_t hi[3], double h, int32_t &x0, int32_t &x1, int32_t &y0,
                                           int32_t &y1) {
    const double N[3] = {(double)v.nx, (double)v.ny, (double)v.nz};
    double pl[3], ph[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pl[a] = fmax((double)lo[a] + h, 0.0);
        ph[a] = fmin((double)hi[a] + 1.0 + h, N[a]);
    }
    double cmin = 1e300, cmax = -1e300, rmin = 1e300, rmax = -1e300;
    bool whole = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double px = (k & 1) ? ph[0] : pl[0], py = (k & 2) ? ph[1] : pl[1], pz = (k & 4) ? ph[2] : pl[2];
        const double vx = px - c.eye[0], vy = py - c.eye[1], vz = pz - c.eye[2];
        double sx = vx * c.r[0] + vy * c.r[1] + vz * c.r[2];
        double sy = vx * c.u[0] + vy * c.u[1] + vz * c.u[2];
        if (c.kind == VR_PERSPECTIVE) {
            const double depth = vx * c.f[0] + vy * c.f[1] + vz * c.f[2];
            if (depth < 1.0) whole = true;
            const double id = 1.0 / fmax(depth, 1e-9);
            sx *= id;
            sy *= id;
        }
        const double col = (sx / c.a + 1.0) * 0.5 * c.W - 0.5;
        const double row = (1.0 - sy / c.b) * 0.5 * c.H - 0.5;
        cmin = fmin(cmin, col); cmax = fmax(cmax, col);
        rmin = fmin(rmin, row); rmax = fmax(rmax, row);
    }
    // Pixel (col, row)'s ray meets the region iff (col, row) lies in the
    // projected hull, whose bounding box this is.  The margin (1/20 pixel)
    // covers the rounding of this projection and the drift of the samples'
    // fixed-point positions from the exact ray (below 2e-6 voxel over the
    // longest ray, under 1/200 pixel once the region is at least one voxel
    // in front of the eye; nearer regions take the whole tile).  Clamp
    // before converting.
    const double lim = 1e9, m = 0.05;
    x0 = whole ? 0 : (int32_t)fmax(floor(fmax(cmin - m, -lim)) - c.tile_x0, 0.0);
    x1 = whole ? c.tile_w : (int32_t)fmin(floor(fmin(cmax + m, lim)) + 1.0 - c.tile_x0, (double)c.tile_w);
    y0 = whole ? 0 : (int32_t)fmax(floor(fmax(rmin - m, -lim)) - c.tile_y0, 0.0);
    y1 = whole ? c.tile_h : (int32_t)fmin(floor(fmin(rmax + m, lim)) + 1.0 - c.tile_y0, (double)c.tile_h);
    if (x1 < x0) x1 = x0;
    if (y1 < y0) y1 = y0;
}

// The voxels of one block, staged through registers.  From the x-fastest
// copy (LINES false): rows of kBX + 1 elements from padded x index jx*kBX, as
// 16-byte chunks (the last chunk of a row clamped to the row's end: its
// clamped voxels are never sampled).  From the line copy (LINES true, FP32):
// one 32-element line per row, line jx of the row, which holds padded x
// indices [31 jx, 31 jx + 31]: 8 chunks of one 128-byte line.  Loads and
// stores are branch-free (a chunk past the box reloads chunk 0 and goes to a
// spare slot), so all loads of a block stay in flight together.
template <typename S, int BY, int BZ, int NT, bool LINES>
struct BlockLoad {
    static constexpr int EPC = 16 / (int)sizeof(S);
    static constexpr int CPR = LINES ? 32 / EPC : (kBX + 1 + EPC - 1) / EPC;
    static constexpr int ROWS = (BY + 1) * (BZ + 1);
    static constexpr int CHUNKS = CPR * ROWS;
    static constexpr int PASSES = (CHUNKS + NT - 1) / NT;
    static constexpr int FLOATS = kPX * ROWS;

    static __device__ __forceinline__ void load(uint4 (&raw)[PASSES], const VolDev &V, int32_t jx, int32_t jy,
                                                int32_t jz, int tid) {
        const int64_t pmax_x = (int64_t)V.Px - EPC;
        const int32_t py_max = V.ny + 1, pz_max = V.nz + 1;
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int c = tid + p * NT;
            const int cc = c < CHUNKS ? c : 0;
            const int row = cc / CPR, ch = cc - row * CPR;
            const int ly = row % (BY + 1), lz = row / (BY + 1);
            const int64_t gy = min(jy * BY + ly, py_max), gz = min(jz * BZ + lz, pz_max);
            if (LINES) {
                const float *lines = (const float *)V.data + V.line_off;
                raw[p] = *(const uint4 *)(lines + ((gz * V.Py + gy) * V.lpr + jx) * 32 + ch * EPC);
            } else {
                const int64_t gx = min((int64_t)jx * kBX + ch * EPC, pmax_x);
                raw[p] = *(const uint4 *)((const S *)V.data + (gz * V.sz + gy * V.sy + gx));
            }
        }
    }
    static __device__ __forceinline__ void store(const uint4 (&raw)[PASSES], float *box, int tid) {
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int c = tid + p * NT;
            const bool in = c < CHUNKS;
            const int cc = in ? c : 0;
            const int row = cc / CPR, ch = cc - row * CPR;
            float *dst = in ? box + row * kPX + ch * EPC : box + FLOATS;
            if (sizeof(S) == 4) {
                const uint4 v = raw[p];
                *(float4 *)dst = make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                                             __uint_as_float(v.w));
            } else {
                const uint32_t w[4] = {raw[p].x, raw[p].y, raw[p].z, raw[p].w};
                float e[8];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (__is_same(S, _Float16)) {
                        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
                        const h2 t = __builtin_bit_cast(h2, w[q]);
                        e[2 * q] = (float)t[0];
                        e[2 * q + 1] = (float)t[1];
                    } else {
                        e[2 * q] = __uint_as_float(w[q] << 16);
                        e[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
                    }
                }
                // a row holds kPX floats: the second half of the last chunk
                // of a row (elements past kPX) is dropped
                *(float4 *)dst = make_float4(e[0], e[1], e[2], e[3]);
                if (!in || ch * EPC + 8 <= kPX) *(float4 *)(dst + 4) = make_float4(e[4], e[5], e[6], e[7]);
            }
        }
    }
};

// Largest of the samples [kb, ke) of ray R in the LDS box of block lo;
// sample kb is at position p.
template <int FILTER, int BX, int BY, int BZ>
__device__ __forceinline__ float block_max(const VolDev &V, const RayRec &R, int32_t kb, int32_t ke,
                                           const int64_t p[3], const int32_t lo[3], const float *box) {
    constexpr uint32_t bM = 4u * kPX, bS = 4u * kPX * (BY + 1);
    // positions relative to the block's low corner: the integer part is then
    // the box index, the fraction is unchanged
    int64_t q0 = p[0] - (int64_t)lo[0] * 4294967296LL, q1 = p[1] - (int64_t)lo[1] * 4294967296LL;
    int64_t q2 = p[2] - (int64_t)lo[2] * 4294967296LL;
    // opaque to the optimizer, which would otherwise keep p as the loop's
    // positions and subtract the corner again at every sample
    asm volatile("" : "+v"(q0), "+v"(q1), "+v"(q2));
    const char *L = (const char *)box;
    float m = -INFINITY;
    for (int32_t k = kb; k < ke; ++k) {
        const int32_t ix = fix_int(q0), iy = fix_int(q1), iz = fix_int(q2);
        // the box holds corner offsets [0, BX] x [0, BY] x [0, BZ]: a sample's low corner is inside the block
        VR_BOUNDS(V, ix >= 0 && iy >= 0 && iz >= 0 && ix < BX && iy < BY && iz < BZ);
        const uint32_t o = (uint32_t)(ix + __mul24(iy, kPX) + __mul24(iz, kPX * (BY + 1))) << 2;
        float s;
        if (FILTER == VR_NEAREST) {
            s = *(const float *)(L + o);
        } else {
            const float fx = fix_frac(q0), fy = fix_frac(q1), fz = fix_frac(q2);
            // one opaque base register for the far plane, so that its four
            // reads pair into two two-element LDS reads off it (the plane's
            // offset exceeds their immediate range)
            uint32_t oz = o + bS;
            asm volatile("" : "+v"(oz));
            const float *pa = (const float *)(L + o), *pb = (const float *)(L + o + bM);
            const float *pc = (const float *)(L + oz), *pd = (const float *)(L + oz + bM);
            const float c000 = pa[0], c100 = pa[1], c010 = pb[0], c110 = pb[1];
            const float c001 = pc[0], c101 = pc[1], c011 = pd[0], c111 = pd[1];
            const float x00 = fmaf(fx, c100 - c000, c000), x10 = fmaf(fx, c110 - c010, c010);
            const float x01 = fmaf(fx, c101 - c001, c001), x11 = fmaf(fx, c111 - c011, c011);
            const float y0 = fmaf(fy, x10 - x00, x00), y1 = fmaf(fy, x11 - x01, x01);
            s = fmaf(fz, y1 - y0, y0);
        }
        // max(m, s) as the bare instruction: both are results of FP
        // arithmetic (or -inf), so the quieting the compiler would add for
        // fmaxf is not needed
        float r;
        asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(s), "v"(m));
        m = r;
        q0 += R.D[0]; q1 += R.D[1]; q2 += R.D[2];
    }
    return m;
}

// The FP32 value of a 64-bit integer below 2^53 in magnitude, rounded once
// (the same value as the plain conversion): both halves and their sum are
// exact in FP64.
__device__ __forceinline__ float i64_to_f32(int64_t v) {
    return (float)fma((double)(int32_t)(v >> 32), 4294967296.0, (double)(uint32_t)v);
}

// The exact run [kb, ke) of samples of R in the corner-index box [lo, hi],
// and the position p of sample kb: per axis a float estimate of where the
// position crosses the box's faces, widened, then trimmed from both ends by
// exact comparisons (the samples in a box form one run, so trimming a run
// that contains them yields them).
__device__ __forceinline__ bool in_box(int64_t x0, int64_t x1, int64_t x2, const int32_t lo[3],
                                       const int32_t hi[3]) {
    const int32_t c0 = fix_int(x0), c1 = fix_int(x1), c2 = fix_int(x2);
    return ((uint32_t)(c0 >= lo[0]) & (uint32_t)(c0 <= hi[0]) & (uint32_t)(c1 >= lo[1]) & (uint32_t)(c1 <= hi[1]) &
            (uint32_t)(c2 >= lo[2]) & (uint32_t)(c2 <= hi[2])) != 0;
}

__device__ __forceinline__ void block_run(const RayRec &R, const int32_t lo[3], const int32_t hi[3], int32_t &kb,
                                          int32_t &ke, int64_t p[3]) {
    kb = 0;
    ke = R.n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t lq = (int64_t)lo[a] * 4294967296LL - R.Q[a];
        const int64_t hq = (int64_t)(hi[a] + 1) * 4294967296LL - R.Q[a];
        if (R.D[a] == 0) {
            if (lq > 0 || hq <= 0) ke = 0;
        } else {
            const float ka = i64_to_f32(lq) * R.rd[a], kc = i64_to_f32(hq) * R.rd[a];
            const float kmn = fminf(fmaxf(fminf(ka, kc), -1e9f), 1e9f);
            const float kmx = fminf(fmaxf(fmaxf(ka, kc), -1e9f), 1e9f);
            kb = max(kb, (int32_t)floorf(kmn) - 1);
            ke = min(ke, (int32_t)ceilf(kmx) + 2);
        }
    }
    p[0] = R.Q[0] + (int64_t)kb * R.D[0];
    p[1] = R.Q[1] + (int64_t)kb * R.D[1];
    p[2] = R.Q[2] + (int64_t)kb * R.D[2];
#pragma clang loop vectorize(disable) interleave(disable) unroll(disable)
    while (kb < ke && !in_box(p[0], p[1], p[2], lo, hi)) {
        ++kb;
        p[0] += R.D[0]; p[1] += R.D[1]; p[2] += R.D[2];
    }
    if (kb < ke) {
        int64_t e0 = R.Q[0] + (int64_t)(ke - 1) * R.D[0];
        int64_t e1 = R.Q[1] + (int64_t)(ke - 1) * R.D[1];
        int64_t e2 = R.Q[2] + (int64_t)(ke - 1) * R.D[2];
#pragma clang loop vectorize(disable) interleave(disable) unroll(disable)
        while (!in_box(e0, e1, e2, lo, hi)) {     // sample kb is inside: stops there at the latest
            --ke;
            e0 -= R.D[0]; e1 -= R.D[1]; e2 -= R.D[2];
        }
    }
}

// A workgroup walks blocks jx of its run along x (at most kMaxRun).  The
// pixel rectangles of the run's blocks are computed first, one block per
// lane, into LDS.  The voxel loads of the next non-empty block are issued
// before the current block is sampled, so their latency hides behind the
// sampling.

template <typename S, int FILTER, int BY, int BZ, int NT, bool LINES>
__global__ __launch_bounds__(NT, (waves_per_simd<BY, BZ, NT>())) void k_mip_blocks(BlockArgs B) {
    using LD = BlockLoad<S, BY, BZ, NT, LINES>;
    constexpr int BX = LINES ? kBXL : kBX;
    __shared__ __align__(16) float box[LD::FLOATS + 8];
    __shared__ int4 rects[kMaxRun];
    const MarchArgs &A = B.m;
    const VolDev &V = A.vol;
    const int tid = threadIdx.x;
    const int32_t rx = (int32_t)(blockIdx.x % (uint32_t)B.runs_x);
    const int32_t jy = (int32_t)((blockIdx.x / (uint32_t)B.runs_x) % (uint32_t)B.nb[1]);
    const int32_t jz = (int32_t)(blockIdx.x / ((uint32_t)B.runs_x * (uint32_t)B.nb[1]));
    const int32_t j0 = rx * B.run, nrun = min(B.run, B.nb[0] - j0);
    const int32_t lo_y = jy * BY - 1, lo_z = jz * BZ - 1;
    if (tid < nrun) {
        const int32_t j = j0 + tid;
        const int32_t lo[3] = {j * BX - 1, lo_y, lo_z};
        const int32_t hi[3] = {lo[0] + BX - 1, lo_y + BY - 1, lo_z + BZ - 1};
        int32_t x0, x1, y0, y1;
        block_rect(A.cam, V, lo, hi, FILTER == VR_TRILINEAR ? 0.5 : 0.0, x0, x1, y0, y1);
        rects[tid] = make_int4(x0, x1, y0, y1);
    }
    __syncthreads();
    // the next block of the run, from t on, with a non-empty rectangle (uniform)
    auto next_block = [&](int32_t t) {
        for (; t < nrun; ++t) {
            const int4 r = rects[t];
            if (r.y > r.x && r.w > r.z) break;
        }
        return t;
    };
    uint32_t *out = (uint32_t *)A.out;
    // pixel i of block t's rectangle
    auto pixel = [&](const int4 &rc, int32_t i) {
        const int32_t fw = rc.y - rc.x, iy = i / fw;
        return (int64_t)(rc.z + iy) * A.cam.tile_w + rc.x + (i - iy * fw);
    };
    auto npix_of = [&](const int4 &rc) { return (rc.y - rc.x) * (rc.w - rc.z); };
    uint4 raw[LD::PASSES];
    RayRec R{};
    int32_t t = next_block(0);
    if (t < nrun) {
        LD::load(raw, V, j0 + t, jy, jz, tid);
        if (tid < npix_of(rects[t])) R = B.tab[pixel(rects[t], tid)];
    }
    while (t < nrun) {
        __syncthreads();                          // the previous block's samples are done
        LD::store(raw, box, tid);
        __syncthreads();
        // the next block: this lane's first ray record, then the voxel loads.
        // Vector loads complete in issue order, so a record load issued after
        // the voxel loads would wait for all of them.
        const int32_t tn = next_block(t + 1);
        RayRec Rn{};
        if (tn < nrun && tid < npix_of(rects[tn])) Rn = B.tab[pixel(rects[tn], tid)];
        asm volatile("" ::: "memory");
        if (tn < nrun) LD::load(raw, V, j0 + tn, jy, jz, tid);
        const int4 rc = rects[t];
        const int32_t lo[3] = {(j0 + t) * BX - 1, lo_y, lo_z};
        const int32_t hi[3] = {lo[0] + BX - 1, lo_y + BY - 1, lo_z + BZ - 1};
        const int32_t npx = npix_of(rc);
        for (int32_t i = tid; i < npx; i += NT) {
            const int64_t pix = pixel(rc, i);
            if (i != tid) R = B.tab[pix];
            int32_t kb, ke;
            int64_t p[3];
            block_run(R, lo, hi, kb, ke, p);
            if (kb < ke) atomicMax(out + pix, mip_enc(block_max<FILTER, BX, BY, BZ>(V, R, kb, ke, p, lo, box)));
        }
        R = Rn;
        t = tn;
    }
}

template <typename S, int FILTER, int BY, int BZ, int NT>
static void launch_blocks_t(const BlockArgs &b, unsigned groups, hipStream_t s) {
    if constexpr (__is_same(S, float)) {
        if (b.m.vol.lpr > 0) {
            hipLaunchKernelGGL((k_mip_blocks<S, FILTER, BY, BZ, NT, true>), dim3(groups), dim3(NT), 0, s, b);
            return;
        }
    }
    hipLaunchKernelGGL((k_mip_blocks<S, FILTER, BY, BZ, NT, false>), dim3(groups), dim3(NT), 0, s, b);
}

template <int BY, int BZ, int NT>
static void launch_blocks_shape(const BlockArgs &b, int32_t dtype, int32_t filter, unsigned groups, hipStream_t s) {
    if (filter == VR_NEAREST) {
        if (dtype == VR_F32) launch_blocks_t<float, VR_NEAREST, BY, BZ, NT>(b, groups, s);
        else if (dtype == VR_F16) launch_blocks_t<_Float16, VR_NEAREST, BY, BZ, NT>(b, groups, s);
        else launch_blocks_t<bf16_t, VR_NEAREST, BY, BZ, NT>(b, groups, s);
    } else {
        if (dtype == VR_F32) launch_blocks_t<float, VR_TRILINEAR, BY, BZ, NT>(b, groups, s);
        else if (dtype == VR_F16) launch_blocks_t<_Float16, VR_TRILINEAR, BY, BZ, NT>(b, groups, s);
        else launch_blocks_t<bf16_t, VR_TRILINEAR, BY, BZ, NT>(b, groups, s);
    }
}

int64_t mip_blocks_workspace(int64_t npix) { return npix * (int64_t)sizeof(RayRec); }

hipError_t launch_mip_blocks(const MarchArgs &a, int32_t filter, void *ws, int32_t run, int32_t shape,
                             hipStream_t s) {
    const VolDev &v = a.vol;
    if (!v.single || v.sx != 1 || run < 1 || run > kMaxRun || !a.out || !ws || shape < 0 || shape > 2)
        return hipErrorInvalidValue;
    const int64_t npix = (int64_t)a.cam.tile_w * a.cam.tile_h;
    if (npix == 0) return hipSuccess;
    RayRec *tab = (RayRec *)ws;
    const unsigned g1 = (unsigned)((npix + 255) / 256);
    if (filter == VR_NEAREST) hipLaunchKernelGGL(k_raytable<VR_NEAREST>, dim3(g1), dim3(256), 0, s, a, tab);
    else hipLaunchKernelGGL(k_raytable<VR_TRILINEAR>, dim3(g1), dim3(256), 0, s, a, tab);
    // block shapes (y, z edges; threads): 0 = 16 x 16, 256; 1 = 32 x 16, 256; 2 = 32 x 16, 512
    const int32_t by = shape == 0 ? 16 : 32, bz = 16;
    BlockArgs b{};
    b.m = a;
    b.tab = tab;
    // blocks cover corner indices [-1, N] of each axis
    // the line copy, when the layout holds one (FP32 with three copies), else the x-fastest copy
    b.nb[0] = (v.lpr > 0 && v.dtype == VR_F32) ? v.lpr : (v.nx + 2 + kBX - 1) / kBX;
    b.nb[1] = (v.ny + 2 + by - 1) / by;
    b.nb[2] = (v.nz + 2 + bz - 1) / bz;
    b.run = run;
    b.runs_x = (b.nb[0] + run - 1) / run;
    const int64_t groups = (int64_t)b.runs_x * b.nb[1] * b.nb[2];
    if (groups > 0x7fffffffLL) return hipErrorInvalidValue;
    if (shape == 0) launch_blocks_shape<16, 16, 256>(b, v.dtype, filter, (unsigned)groups, s);
    else if (shape == 1) launch_blocks_shape<32, 16, 256>(b, v.dtype, filter, (unsigned)groups, s);
    else launch_blocks_shape<32, 16, 512>(b, v.dtype, filter, (unsigned)groups, s);
    hipLaunchKernelGGL(k_mip_decode, dim3(g1), dim3(256), 0, s, (uint32_t *)a.out, npix);
    return hipGetLastError();
}

}  // namespace vr
