// k_transcode.hip -- K0: float32 (z,y,x) cube -> brick-major layout with a
// one-voxel apron, optionally narrowed to FP16/BF16 with round-to-nearest-even.
//
// One 64-lane wave writes one destination row (Px voxels of one brick plane);
// reads and writes are both contiguous along x.  HBM-bound: 4 bytes read and
// storage-size bytes written per destination voxel.
#include "vr_internal.h"

namespace vr {

__device__ __forceinline__ void put(float *p, float v) { *p = v; }
__device__ __forceinline__ void put(_Float16 *p, float v) { *p = (_Float16)v; }
__device__ __forceinline__ void put(bf16_t *p, float v) {
    uint32_t u = __float_as_uint(v);
    uint16_t h;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        h = (uint16_t)((u >> 16) | 0x40u);        // quiet NaN
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);           // round to nearest, ties to even
        h = (uint16_t)(u >> 16);
    }
    p->bits = h;
}

template <typename S>
__global__ __launch_bounds__(256) void k_transcode(const float *__restrict__ src, VolDev v,
                                                   int64_t z0, int64_t z1, int64_t bz_lo,
                                                   int64_t rows_total) {
    int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= rows_total) return;
    int lane = threadIdx.x & 63;
    // row -> (brick in the z-layer range, lz, ly)
    int64_t ly = row % v.Py;
    int64_t t = row / v.Py;
    int64_t lz = t % v.Pz;
    int64_t bl = t / v.Pz;                         // brick index relative to layer bz_lo
    int64_t bx = bl % v.nbx;
    int64_t by = (bl / v.nbx) % v.nby;
    int64_t bz = bz_lo + bl / ((int64_t)v.nbx * v.nby);
    int64_t gz = bz * v.Bz - 1 + lz;
    gz = gz < 0 ? 0 : (gz > v.nz - 1 ? v.nz - 1 : gz);
    if (gz < z0 || gz >= z1) return;
    int64_t gy = by * v.By - 1 + ly;
    gy = gy < 0 ? 0 : (gy > v.ny - 1 ? v.ny - 1 : gy);
    const float *srow = src + ((gz - z0) * v.ny + gy) * (int64_t)v.nx;
    int64_t brick = (bz * v.nby + by) * v.nbx + bx;
    S *drow = (S *)v.data + brick * v.brick_elems + (lz * v.Py + ly) * (int64_t)v.Px;
    int64_t xo = bx * v.Bx - 1;
    for (int lx = lane; lx < v.Px; lx += 64) {
        int64_t gx = xo + lx;
        gx = gx < 0 ? 0 : (gx > v.nx - 1 ? v.nx - 1 : gx);
        put(drow + lx, srow[gx]);
    }
}

// Copy ORI (1: y fastest, then z, x; 2: z fastest, then x, y) of a one-brick
// layout, through a 64 x 64 LDS tile: reads run along x (the source's
// storage order), writes along the copy's fastest axis.  One workgroup per
// tile of (fastest axis f) x (x) at one value of the third axis t.  Indices
// are padded (0 .. n+1, clamped to the cube); only source planes z in
// [z0, z1) are written.
template <typename S, int ORI>
__global__ __launch_bounds__(256) void k_transcode_t(const float *__restrict__ src, VolDev v, S *__restrict__ dst,
                                                     int64_t z0, int64_t z1) {
    __shared__ float tile[64][65];
    constexpr int AF = ORI, AM = (ORI + 1) % 3, AS = (ORI + 2) % 3;
    constexpr int AT = ORI == 1 ? 2 : 1;              // the axis that is neither f nor x
    const int64_t n[3] = {v.nx, v.ny, v.nz};
    int64_t pf, pm, ps;
    copy_pitches(v, ORI, pf, pm, ps);
    const int64_t f0 = (int64_t)blockIdx.x * 64, x0 = (int64_t)blockIdx.y * 64, lt = blockIdx.z;
    const int tid = threadIdx.x;
    auto clampi = [](int64_t i, int64_t hi) { return i < 0 ? 0 : (i > hi ? hi : i); };
    // read: rows of x at 64 values of f
    for (int i = 0; i < 16; ++i) {
        const int r = (tid >> 6) + 4 * i, c = tid & 63;
        int64_t l[3];
        l[AF] = f0 + r;
        l[0] = x0 + c;
        l[AT] = lt;
        int64_t g[3];
        for (int a = 0; a < 3; ++a) g[a] = clampi(l[a] - 1, n[a] - 1);
        float val = 0.0f;
        if (g[2] >= z0 && g[2] < z1) val = src[((g[2] - z0) * n[1] + g[1]) * n[0] + g[0]];
        tile[r][c] = val;
    }
    __syncthreads();
    // write: rows along f at 64 values of x
    for (int i = 0; i < 16; ++i) {
        const int c = (tid >> 6) + 4 * i, r = tid & 63;
        int64_t l[3];
        l[AF] = f0 + r;
        l[0] = x0 + c;
        l[AT] = lt;
        if (l[AF] >= pf || l[0] >= n[0] + 2) continue;
        const int64_t gz = clampi(l[2] - 1, n[2] - 1);
        if (gz < z0 || gz >= z1) continue;
        put(dst + (l[AS] * pm + l[AM]) * pf + l[AF], tile[r][c]);
    }
}

template <typename S>
static hipError_t launch_copies(const float *src, const VolDev &v, int64_t z0, int64_t z1, hipStream_t s) {
    for (int c = 1; c < 3; ++c) {
        int64_t pf, pm, ps;
        copy_pitches(v, c, pf, pm, ps);
        const int64_t nx2 = v.nx + 2;
        const int64_t nt = (c == 1 ? v.nz : v.ny) + 2;
        dim3 g((unsigned)((pf + 63) / 64), (unsigned)((nx2 + 63) / 64), (unsigned)nt), b(256);
        S *dst = (S *)v.data + v.copy_off[c];
        if (c == 1) hipLaunchKernelGGL((k_transcode_t<S, 1>), g, b, 0, s, src, v, dst, z0, z1);
        else hipLaunchKernelGGL((k_transcode_t<S, 2>), g, b, 0, s, src, v, dst, z0, z1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_transcode(const float *src, const VolDev &v, int64_t z0, int64_t z1, hipStream_t s) {
    // brick z-layers whose stored planes (with apron) touch [z0, z1)
    int64_t bz_lo = (z0 - 1) >= 0 ? (z0 - 1) / v.Bz : 0;
    int64_t bz_hi = z1 / v.Bz;                      // inclusive
    if (bz_lo > v.nbz - 1) bz_lo = v.nbz - 1;
    if (bz_hi > v.nbz - 1) bz_hi = v.nbz - 1;
    int64_t layers = bz_hi - bz_lo + 1;
    int64_t rows = layers * v.nbx * v.nby * (int64_t)v.Pz * v.Py;
    int64_t blocks = (rows + 3) / 4;
    if (blocks <= 0) return hipSuccess;
    dim3 g((unsigned)blocks), b(256);
    switch (v.dtype) {
        case VR_F32: hipLaunchKernelGGL(k_transcode<float>, g, b, 0, s, src, v, z0, z1, bz_lo, rows); break;
        case VR_F16: hipLaunchKernelGGL(k_transcode<_Float16>, g, b, 0, s, src, v, z0, z1, bz_lo, rows); break;
        default: hipLaunchKernelGGL(k_transcode<bf16_t>, g, b, 0, s, src, v, z0, z1, bz_lo, rows); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || v.orients < 3) return e;
    switch (v.dtype) {
        case VR_F32: return launch_copies<float>(src, v, z0, z1, s);
        case VR_F16: return launch_copies<_Float16>(src, v, z0, z1, s);
        default: return launch_copies<bf16_t>(src, v, z0, z1, s);
    }
}

}  // namespace vr
