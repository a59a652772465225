// k_backward.hip -- K5: adjoint of the composite render with respect to the
// transfer-function table and the voxels.
//
// The forward pass (k_march / k_slab with save_for_backward) stored, per
// pixel, the number of samples taken m and the transmittance in front of
// samples 0, kCkpt, 2 kCkpt, ... (segment checkpoints), so no per-sample
// state is kept.  Here one lane owns one ray and walks its segments from the
// last to the first: it replays the kCkpt samples of a segment forward from
// the checkpoint into registers (the transmittance in front of each sample
// and the sample value, with the forward's own arithmetic), then walks them
// backwards carrying the suffix sums
//   S (colour behind the sample, as seen from it) and P (transmittance behind):
//   dL/dc_k = gC T_k a_k,   dL/da_k = T_k [gC.(c_k - S) + gA P],
//   S <- a_k c_k + (1 - a_k) S,   P <- (1 - a_k) P,
// then chains through the table's linear interpolation (LDS-privatised table
// gradient, flushed once per workgroup) and the trilinear weights (corners
// clamped to the cube as the clamp-to-edge sampling does; a lane sums the
// contributions of its consecutive samples in one cell first, and when the
// ray steps into a neighbouring cell the four sums of the shared face stay in
// registers).  Each sample
// is gathered once; the only LDS are the table, its gradient and the voxel
// cache below, which keeps several workgroups per CU to hide the gathers.
//
// Voxel gradients are privatised per workgroup in an LDS cache: a
// direct-mapped table of kCache voxel slots (tag = voxel index, value = the
// workgroup's partial sum); an empty slot is claimed with an LDS
// compare-and-swap, and a contribution whose slot already holds another
// voxel goes straight to memory.  The workgroup's rays are neighbours (a
// compact tile of the image, lanes kStride pixels apart), so they revisit the
// same voxels many times, and each cached voxel costs one atomic in memory
// when the workgroup ends instead of one per ray and cell.
#include "vr_internal.h"

namespace vr {

constexpr int kSeg = kCkpt;     // samples per checkpoint segment, replayed into registers
constexpr int kBackThreads = 128;
// Lanes of a workgroup take pixels kStride apart in x and y (16 x 8 lanes
// over a (16 kStride) x (8 kStride) super-tile; the kStride^2 workgroups of a
// super-tile take the offsets): the workgroup's rays stay close enough to
// share voxels in its cache, and lanes of one LDS atomic rarely hit the same
// address.
constexpr int kStride = 2;
constexpr int kCache = 2048;    // voxel slots per workgroup (power of two; 16 KiB of LDS)
constexpr int kCacheBits = __builtin_ctz(kCache);
constexpr uint32_t kEmpty = 0xffffffffu;

// Add g to voxel v of the gradient through the workgroup's cache (nv < 2^32
// - 1 voxels), or straight to memory when v's slot holds another voxel.
__device__ __forceinline__ void cache_add(uint32_t *tag, float *val, float *gv, uint32_t v, float g) {
    const uint32_t h = (v * 2654435761u) >> (32 - kCacheBits);   // multiplicative hash onto kCache slots
    // a slot's tag is set once and never changes: a plain read settles hits
    // and misses on a taken slot, the compare-and-swap only claims an empty one
    uint32_t t = __hip_atomic_load(&tag[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (t == kEmpty) {
        const uint32_t old = atomicCAS(&tag[h], kEmpty, v);
        t = old == kEmpty ? v : old;
    }
    if (t == v) atomicAdd(&val[h], g);
    else unsafeAtomicAdd(gv + v, g);
}

__global__ __launch_bounds__(kBackThreads) void k_backward(BackArgs B) {
    extern __shared__ float smem[];
    const MarchArgs &A = B.m;
    const int n_l = A.lut.n;
    float4 *lut = (float4 *)smem;                        // n_l entries
    float *glut = smem + 4 * n_l;                        // n_l * 4 partial gradients
    uint32_t *ctag = (uint32_t *)(glut + 4 * n_l);      // voxel-gradient cache
    float *cval = (float *)(ctag + kCache);
    const int tid = threadIdx.x;
    for (int i = tid; i < n_l; i += blockDim.x) {
        lut[i] = A.lut.rgba[i];
        glut[4 * i] = glut[4 * i + 1] = glut[4 * i + 2] = glut[4 * i + 3] = 0.0f;
    }
    for (int i = tid; i < kCache; i += blockDim.x) {
        ctag[i] = kEmpty;
        cval[i] = 0.0f;
    }
    __syncthreads();
    const bool cached = (int64_t)A.vol.nx * A.vol.ny * A.vol.nz < (int64_t)kEmpty;

    const int64_t npix = (int64_t)A.cam.tile_w * A.cam.tile_h;
    const int32_t sgx = (A.cam.tile_w + 16 * kStride - 1) / (16 * kStride);
    const int32_t st = (int32_t)blockIdx.x / (kStride * kStride), sub = (int32_t)blockIdx.x % (kStride * kStride);
    const int px = (st % sgx) * 16 * kStride + sub % kStride + kStride * (tid % 16);
    const int py = (st / sgx) * (kBackThreads / 16) * kStride + sub / kStride + kStride * (tid / 16);
    const bool inside = px < A.cam.tile_w && py < A.cam.tile_h;
    const int64_t pix = (int64_t)py * A.cam.tile_w + px;
    const VolDev &V = A.vol;
    int32_t m = 0;
    if (inside) m = A.taken[pix];
    if (m > 0) {
        Ray r{};
        make_ray(A.cam, V, A.cam.tile_x0 + px, A.cam.tile_y0 + py, A.step, r);
        int64_t Q0[3], D[3];
        fix_start(r, A.step, 0, 0.5, Q0, D);
        const float4 g = B.gout[pix];
        float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f, P = 1.0f;
        const int nx = V.nx, ny = V.ny, nz = V.nz;
        const bool use_log = A.trans == 1 || (A.trans == 2 && r.n > 1024);
        // voxel gradients of consecutive samples in the same cell are summed
        // per lane and added to memory once the ray leaves the cell (the
        // step is half a voxel: a cell holds two or three samples of a ray)
        int32_t cx = INT32_MIN, cy = 0, cz = 0;
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        auto flush = [&](uint32_t keep) {
            if (cx == INT32_MIN) return;
            const int X0 = min(max(cx, 0), nx - 1), X1 = min(max(cx + 1, 0), nx - 1);
            const int Y0 = min(max(cy, 0), ny - 1), Y1 = min(max(cy + 1, 0), ny - 1);
            const int Z0 = min(max(cz, 0), nz - 1), Z1 = min(max(cz + 1, 0), nz - 1);
            float *gv = B.grad_vol;
            const int64_t r00 = ((int64_t)Z0 * ny + Y0) * nx, r10 = ((int64_t)Z0 * ny + Y1) * nx;
            const int64_t r01 = ((int64_t)Z1 * ny + Y0) * nx, r11 = ((int64_t)Z1 * ny + Y1) * nx;
            const int64_t at[8] = {r00 + X0, r00 + X1, r10 + X0, r10 + X1, r01 + X0, r01 + X1, r11 + X0, r11 + X1};
            if (cached) {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (!((keep >> i) & 1u) && acc[i] != 0.0f) cache_add(ctag, cval, gv, (uint32_t)at[i], acc[i]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (!((keep >> i) & 1u)) unsafeAtomicAdd(gv + at[i], acc[i]);
            }
        };
        // corner i of a cell is (x, y, z) offset (i & 1, (i >> 1) & 1, i >> 2).
        // Moving to the next cell along one axis keeps the shared face's four
        // sums in registers: they carry over to the new cell's opposite face,
        // and only the other four leave.
        auto move_cell = [&](int ix, int iy, int iz) {
            int axis = -1, dir = 0;
            if (cx != INT32_MIN) {
                const int ddx = ix - cx, ddy = iy - cy, ddz = iz - cz;
                if (ddy == 0 && ddz == 0 && (ddx == 1 || ddx == -1)) { axis = 0; dir = ddx; }
                else if (ddx == 0 && ddz == 0 && (ddy == 1 || ddy == -1)) { axis = 1; dir = ddy; }
                else if (ddx == 0 && ddy == 0 && (ddz == 1 || ddz == -1)) { axis = 2; dir = ddz; }
            }
            // the kept face: the far one (bit set) when moving up, else the near one
            const uint32_t face[3][2] = {{0x55u, 0xAAu}, {0x33u, 0xCCu}, {0x0Fu, 0xF0u}};
            flush(axis < 0 ? 0u : face[axis][dir > 0 ? 1 : 0]);
            auto carry = [&](int lo_i, int hi_i, bool up) {   // corners differing in the axis bit
                if (up) { acc[lo_i] = acc[hi_i]; acc[hi_i] = 0.0f; }
                else { acc[hi_i] = acc[lo_i]; acc[lo_i] = 0.0f; }
            };
            if (axis == 0) { carry(0, 1, dir > 0); carry(2, 3, dir > 0); carry(4, 5, dir > 0); carry(6, 7, dir > 0); }
            else if (axis == 1) { carry(0, 2, dir > 0); carry(1, 3, dir > 0); carry(4, 6, dir > 0); carry(5, 7, dir > 0); }
            else if (axis == 2) { carry(0, 4, dir > 0); carry(1, 5, dir > 0); carry(2, 6, dir > 0); carry(3, 7, dir > 0); }
            else {
#pragma unroll
                for (int i2 = 0; i2 < 8; ++i2) acc[i2] = 0.0f;
            }
            cx = ix; cy = iy; cz = iz;
        };
        for (int seg = (m - 1) / kSeg; seg >= 0; --seg) {
            {
                // replay of the segment from its checkpoint into registers
                // (transmittance in front of each sample and the sample value),
                // then the backward sweep over it
                const int j0 = seg * kSeg, nj = min(kSeg, m - j0);
                float Tj = A.ckpt[(int64_t)seg * npix + pix];
                LogTrans lj;
                if (use_log) lj.L = Tj > 0.0f ? __builtin_amdgcn_logf(Tj) : -INFINITY;
                float Ts[kSeg], ss[kSeg];
                int64_t q0 = Q0[0] + (int64_t)j0 * D[0], q1 = Q0[1] + (int64_t)j0 * D[1],
                        q2 = Q0[2] + (int64_t)j0 * D[2];
#pragma unroll
                for (int i = 0; i < kSeg; ++i) {
                    if (i < nj) {
                        Ts[i] = Tj;
                        ss[i] = gsample<float, VR_TRILINEAR>(V, fix_int(q0), fix_int(q1), fix_int(q2), fix_frac(q0),
                                                             fix_frac(q1), fix_frac(q2));
                        const float a = lut_eval(lut, n_l, A.lut.vmin, A.lut.scale, ss[i]).w;
                        Tj = use_log ? lj.step(a) : Tj - Tj * a;
                        q0 += D[0]; q1 += D[1]; q2 += D[2];
                    }
                }
#pragma unroll
                for (int i = kSeg - 1; i >= 0; --i) {
                    if (i >= nj) continue;
                    q0 -= D[0]; q1 -= D[1]; q2 -= D[2];
                    const int ix = fix_int(q0), iy = fix_int(q1), iz = fix_int(q2);
                    const float fx = fix_frac(q0), fy = fix_frac(q1), fz = fix_frac(q2);
                    const float s = ss[i];
                    // table entry and slope
                    float x = (s - A.lut.vmin) * A.lut.scale;
                    const bool clamped = !(x > 0.0f && x < (float)(n_l - 1));
                    x = fminf(fmaxf(x, 0.0f), (float)(n_l - 1));
                    const int j = min((int)x, n_l - 2);
                    const float w = x - (float)j;
                    const float4 La = lut[j], Lb = lut[j + 1];
                    const bool blank = !(s == s);              // NaN: transparent, uses no table entry
                    const float c0 = fmaf(w, Lb.x - La.x, La.x), c1 = fmaf(w, Lb.y - La.y, La.y);
                    const float c2 = fmaf(w, Lb.z - La.z, La.z), a = blank ? 0.0f : fmaf(w, Lb.w - La.w, La.w);
                    const float Tk = Ts[i];
                    const float ta = Tk * a;
                    const float d0 = g.x * ta, d1 = g.y * ta, d2 = g.z * ta;
                    const float da = Tk * (g.x * (c0 - S0) + g.y * (c1 - S1) + g.z * (c2 - S2) + g.w * P);
                    // table gradient (LDS-privatised)
                    if (B.grad_lut && !blank) {
                        const float wa = 1.0f - w;
                        atomicAdd(&glut[4 * j + 0], wa * d0);
                        atomicAdd(&glut[4 * j + 1], wa * d1);
                        atomicAdd(&glut[4 * j + 2], wa * d2);
                        atomicAdd(&glut[4 * j + 3], wa * da);
                        atomicAdd(&glut[4 * j + 4], w * d0);
                        atomicAdd(&glut[4 * j + 5], w * d1);
                        atomicAdd(&glut[4 * j + 6], w * d2);
                        atomicAdd(&glut[4 * j + 7], w * da);
                    }
                    // value gradient through the table, then the trilinear weights
                    if (B.grad_vol && !clamped) {
                        const float gs = (d0 * (Lb.x - La.x) + d1 * (Lb.y - La.y) + d2 * (Lb.z - La.z) +
                                          da * (Lb.w - La.w)) * A.lut.scale;
                        if (gs != 0.0f) {
                            if (ix != cx || iy != cy || iz != cz) move_cell(ix, iy, iz);
                            const float wx1 = fx, wx0 = 1.0f - fx, wy1 = fy, wy0 = 1.0f - fy, wz1 = fz, wz0 = 1.0f - fz;
                            const float g00 = gs * wz0 * wy0, g10 = gs * wz0 * wy1;
                            const float g01 = gs * wz1 * wy0, g11 = gs * wz1 * wy1;
                            acc[0] = fmaf(g00, wx0, acc[0]);
                            acc[1] = fmaf(g00, wx1, acc[1]);
                            acc[2] = fmaf(g10, wx0, acc[2]);
                            acc[3] = fmaf(g10, wx1, acc[3]);
                            acc[4] = fmaf(g01, wx0, acc[4]);
                            acc[5] = fmaf(g01, wx1, acc[5]);
                            acc[6] = fmaf(g11, wx0, acc[6]);
                            acc[7] = fmaf(g11, wx1, acc[7]);
                        }
                    }
                    S0 = fmaf(a, c0 - S0, S0);
                    S1 = fmaf(a, c1 - S1, S1);
                    S2 = fmaf(a, c2 - S2, S2);
                    P = P - a * P;
                }
            }
        }
        if (B.grad_vol) flush(0u);
    }
    __syncthreads();
    if (B.grad_lut) {
        for (int i = tid; i < 4 * n_l; i += blockDim.x)
            if (glut[i] != 0.0f) unsafeAtomicAdd(B.grad_lut + i, glut[i]);
    }
    if (B.grad_vol && cached) {
        for (int i = tid; i < kCache; i += blockDim.x)
            if (ctag[i] != kEmpty && cval[i] != 0.0f) unsafeAtomicAdd(B.grad_vol + ctag[i], cval[i]);
    }
}

hipError_t launch_backward(const BackArgs &a, hipStream_t s) {
    const int64_t sgx = (a.m.cam.tile_w + 16 * kStride - 1) / (16 * kStride);
    const int64_t sgy = (a.m.cam.tile_h + (kBackThreads / 16) * kStride - 1) / ((kBackThreads / 16) * kStride);
    const unsigned blocks = (unsigned)(sgx * sgy * kStride * kStride);
    const size_t lds = (size_t)a.m.lut.n * 32 + (size_t)kCache * 8;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_backward, dim3(blocks), dim3(kBackThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace vr
