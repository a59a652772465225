// k_transcode.hip -- K0: float32 (z,y,x) cube -> brick-major layout with a
// one-voxel apron, optionally narrowed to FP16/BF16 with round-to-nearest-even,
// and for one-brick layouts the two transposed orientation copies.
// HBM-bound: 4 bytes read and storage-size bytes written per destination
// voxel of each copy.
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

// Four voxels from storage-order FP32 into the layout's storage type.
__device__ __forceinline__ void put4(float *p, float4 v) { *(float4 *)p = v; }
__device__ __forceinline__ void put4(_Float16 *p, float4 v) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    h4 h = {(_Float16)v.x, (_Float16)v.y, (_Float16)v.z, (_Float16)v.w};
    *(h4 *)p = h;
}
__device__ __forceinline__ void put4(bf16_t *p, float4 v) {
    put(p, v.x); put(p + 1, v.y); put(p + 2, v.z); put(p + 3, v.w);
}

// Copy 0 (x fastest, brick-major): a wave writes one destination row (Px
// voxels of one brick plane), four consecutive voxels per lane and step
// (16-byte loads of the source row where all four are inside it, clamped
// scalar loads at the cube's x faces; 16- or 8-byte stores, aligned since Px
// and the brick size are multiples of 8).  Grid: x = groups of 4 rows of a
// plane, y = plane lz, z = brick of the layer range (launched in chunks of
// at most 65535 planes and bricks): no index division per row.
template <typename S>
__global__ __launch_bounds__(256) void k_transcode(const float *__restrict__ src, VolDev v, int32_t z0, int32_t z1,
                                                   int32_t bz_lo, int32_t lz0, int32_t bl0) {
    const int32_t ly = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    if (ly >= v.Py) return;
    const int32_t lz = lz0 + (int32_t)blockIdx.y, bl = bl0 + (int32_t)blockIdx.z;
    const int32_t bxy = v.nbx * v.nby;
    const int32_t bz = bz_lo + bl / bxy, bxy_i = bl - (bl / bxy) * bxy;
    const int32_t by = bxy_i / v.nbx, bx = bxy_i - by * v.nbx;
    const int32_t gz = min(max(bz * v.Bz - 1 + lz, 0), v.nz - 1);
    if (gz < z0 || gz >= z1) return;
    const int32_t gy = min(max(by * v.By - 1 + ly, 0), v.ny - 1);
    const float *srow = src + ((int64_t)(gz - z0) * v.ny + gy) * (int64_t)v.nx;
    const int64_t brick = ((int64_t)bz * v.nby + by) * v.nbx + bx;
    S *drow = (S *)v.data + brick * v.brick_elems + ((int64_t)lz * v.Py + ly) * (int64_t)v.Px;
    const int32_t xo = bx * v.Bx - 1, lane = (int32_t)(threadIdx.x & 63), nx1 = v.nx - 1;
    for (int32_t lx = 4 * lane; lx < v.Px; lx += 256) {
        const int32_t g0 = xo + lx;
        float4 val;
        if (g0 >= 0 && g0 + 3 <= nx1) {
            __builtin_memcpy(&val, srow + g0, 16);
        } else {
            val.x = srow[min(max(g0, 0), nx1)];
            val.y = srow[min(max(g0 + 1, 0), nx1)];
            val.z = srow[min(max(g0 + 2, 0), nx1)];
            val.w = srow[min(max(g0 + 3, 0), nx1)];
        }
        put4(drow + lx, val);
    }
}

// Copy ORI (1: y fastest, then z, x; 2: z fastest, then x, y) of a one-brick
// layout, through a 64 x 64 LDS tile: reads run along x (the source's
// storage order), writes along the copy's fastest axis.  One workgroup per
// tile of (fastest axis f) x (x) at one value of the third axis t.  Indices
// are padded (0 .. n+1, clamped to the cube); only source planes z in
// [z0, z1) are written.  Each thread's 16 reads and 16 writes differ by a
// fixed stride, so the index arithmetic is one addition per element.
template <typename S, int ORI>
__global__ __launch_bounds__(256) void k_transcode_t(const float *__restrict__ src, VolDev v, S *__restrict__ dst,
                                                     int32_t z0, int32_t z1, int32_t t0) {
    __shared__ float tile[64][65];
    int64_t pf, pm, ps;
    copy_pitches(v, ORI, pf, pm, ps);
    const int32_t f0 = (int32_t)blockIdx.x * 64, x0 = (int32_t)blockIdx.y * 64, lt = t0 + (int32_t)blockIdx.z;
    const int32_t tid = (int32_t)threadIdx.x, w4 = tid >> 6, c64 = tid & 63;
    const int32_t nx = v.nx, ny = v.ny, nz = v.nz;
    auto clampi = [](int32_t i, int32_t hi) { return i < 0 ? 0 : (i > hi ? hi : i); };
    // read: row r = w4 + 4 i of the tile holds x = x0 + c64 at f = f0 + r
    {
        const int32_t gx = clampi(x0 + c64 - 1, nx - 1);
        if (ORI == 1) {                                // f = y, t = z
            const int32_t gz = clampi(lt - 1, nz - 1);
            const bool zin = gz >= z0 && gz < z1;
            const float *base = src + (int64_t)(gz - z0) * ny * nx + gx;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int32_t r = w4 + 4 * i;
                const int32_t gy = clampi(f0 + r - 1, ny - 1);
                tile[r][c64] = zin ? base[(int64_t)gy * nx] : 0.0f;
            }
        } else {                                       // f = z, t = y
            const int32_t gy = clampi(lt - 1, ny - 1);
            const float *base = src + (int64_t)gy * nx + gx;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int32_t r = w4 + 4 * i;
                const int32_t gz = clampi(f0 + r - 1, nz - 1);
                tile[r][c64] = (gz >= z0 && gz < z1) ? base[(int64_t)(gz - z0) * ny * nx] : 0.0f;
            }
        }
    }
    __syncthreads();
    // write: tile column c = w4 + 4 i (x = x0 + c) along f = f0 + c64
    const int32_t lf = f0 + c64;
    if (lf >= pf) return;
    if (ORI == 1) {                                    // (x, z, y): x slowest, z middle
        if (clampi(lt - 1, nz - 1) < z0 || clampi(lt - 1, nz - 1) >= z1) return;
        S *d = dst + ((int64_t)x0 * pm + lt) * pf + lf;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int32_t c = w4 + 4 * i;
            if (x0 + c < nx + 2) put(d + (int64_t)c * pm * pf, tile[c64][c]);
        }
    } else {                                           // (y, x, z): y slowest, x middle
        const int32_t gz = clampi(lf - 1, nz - 1);
        if (gz < z0 || gz >= z1) return;
        S *d = dst + ((int64_t)lt * pm + x0) * pf + lf;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int32_t c = w4 + 4 * i;
            if (x0 + c < nx + 2) put(d + (int64_t)c * pf, tile[c64][c]);
        }
    }
}

template <typename S>
static hipError_t launch_copies(const float *src, const VolDev &v, int64_t z0, int64_t z1, hipStream_t s) {
    for (int c = 1; c < 3; ++c) {
        int64_t pf, pm, ps;
        copy_pitches(v, c, pf, pm, ps);
        const int64_t nx2 = v.nx + 2;
        const int64_t nt = (c == 1 ? v.nz : v.ny) + 2;
        S *dst = (S *)v.data + v.copy_off[c];
        for (int64_t t0 = 0; t0 < nt; t0 += 65535) {       // grid z holds at most 65535 planes
            dim3 g((unsigned)((pf + 63) / 64), (unsigned)((nx2 + 63) / 64), (unsigned)(nt - t0 < 65535 ? nt - t0 : 65535)),
                b(256);
            const int32_t a = (int32_t)z0, e1 = (int32_t)z1, t = (int32_t)t0;
            if (c == 1) hipLaunchKernelGGL((k_transcode_t<S, 1>), g, b, 0, s, src, v, dst, a, e1, t);
            else hipLaunchKernelGGL((k_transcode_t<S, 2>), g, b, 0, s, src, v, dst, a, e1, t);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// The line copy (FP32 three-copy layouts): padded row (lz, ly) cut into
// lines of 32 elements, element e of line L = padded x index 31 L + e,
// clamped to the row's last index.  One thread per element; blockIdx.y is the
// padded row within the plane, blockIdx.z the padded plane from lz0.  Only
// planes whose source plane lies in [z0, z1) are written.
__global__ __launch_bounds__(256) void k_transcode_lines(const float *__restrict__ src, VolDev v,
                                                         float *__restrict__ dst, int32_t z0, int32_t z1,
                                                         int32_t ly0, int32_t lz0) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row_elems = (int64_t)v.lpr * 32;
    if (e >= row_elems) return;
    const int32_t ly = ly0 + (int32_t)blockIdx.y, lz = lz0 + (int32_t)blockIdx.z;
    const int32_t nx = v.nx, ny = v.ny, nz = v.nz;
    auto clampi = [](int64_t i, int32_t hi) { return (int32_t)(i < 0 ? 0 : (i > hi ? hi : i)); };
    const int32_t gz = clampi(lz - 1, nz - 1);
    if (gz < z0 || gz >= z1) return;
    const int32_t gy = clampi(ly - 1, ny - 1);
    const int64_t L = e >> 5, px = 31 * L + (e & 31);                 // padded x index
    const int32_t gx = clampi(min(px, (int64_t)nx + 1) - 1, nx - 1);
    dst[((int64_t)lz * v.Py + ly) * row_elems + e] = src[((int64_t)(gz - z0) * ny + gy) * nx + gx];
}

hipError_t launch_transcode(const float *src, const VolDev &v, int64_t z0, int64_t z1, hipStream_t s) {
    // brick z-layers whose stored planes (with apron) touch [z0, z1)
    int64_t bz_lo = (z0 - 1) >= 0 ? (z0 - 1) / v.Bz : 0;
    int64_t bz_hi = z1 / v.Bz;                      // inclusive
    if (bz_lo > v.nbz - 1) bz_lo = v.nbz - 1;
    if (bz_hi > v.nbz - 1) bz_hi = v.nbz - 1;
    const int64_t bricks = (bz_hi - bz_lo + 1) * v.nbx * v.nby;
    if (bricks <= 0) return hipSuccess;
    const int32_t a = (int32_t)z0, c = (int32_t)z1, l = (int32_t)bz_lo;
    constexpr int64_t kMaxGrid = 65535;
    for (int64_t lz0 = 0; lz0 < v.Pz; lz0 += kMaxGrid)
        for (int64_t bl0 = 0; bl0 < bricks; bl0 += kMaxGrid) {
            dim3 g((unsigned)((v.Py + 3) / 4), (unsigned)(v.Pz - lz0 < kMaxGrid ? v.Pz - lz0 : kMaxGrid),
                   (unsigned)(bricks - bl0 < kMaxGrid ? bricks - bl0 : kMaxGrid)), b(256);
            const int32_t p = (int32_t)lz0, q = (int32_t)bl0;
            switch (v.dtype) {
                case VR_F32: hipLaunchKernelGGL(k_transcode<float>, g, b, 0, s, src, v, a, c, l, p, q); break;
                case VR_F16: hipLaunchKernelGGL(k_transcode<_Float16>, g, b, 0, s, src, v, a, c, l, p, q); break;
                default: hipLaunchKernelGGL(k_transcode<bf16_t>, g, b, 0, s, src, v, a, c, l, p, q); break;
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    if (v.orients < 3) return hipSuccess;
    hipError_t e;
    switch (v.dtype) {
        case VR_F32: e = launch_copies<float>(src, v, z0, z1, s); break;
        case VR_F16: e = launch_copies<_Float16>(src, v, z0, z1, s); break;
        default: e = launch_copies<bf16_t>(src, v, z0, z1, s); break;
    }
    if (e != hipSuccess || v.lpr <= 0 || v.dtype != VR_F32) return e;
    // padded planes whose source plane lies in [z0, z1): z + 1 for z in the
    // slab, plus the apron planes 0 and nz + 1 with the first and last slab
    const int64_t lz_lo = z0 == 0 ? 0 : z0 + 1, lz_hi = z1 == v.nz ? (int64_t)v.nz + 1 : z1;
    float *dst = (float *)v.data + v.line_off;
    const unsigned gxb = (unsigned)(((int64_t)v.lpr * 32 + 255) / 256);
    for (int64_t lz = lz_lo; lz <= lz_hi; lz += 65535)
        for (int64_t ly = 0; ly < v.Py; ly += 65535) {
            dim3 g(gxb, (unsigned)(v.Py - ly < 65535 ? v.Py - ly : 65535),
                   (unsigned)(lz_hi + 1 - lz < 65535 ? lz_hi + 1 - lz : 65535)),
                b(256);
            hipLaunchKernelGGL(k_transcode_lines, g, b, 0, s, src, v, dst, (int32_t)z0, (int32_t)z1, (int32_t)ly,
                               (int32_t)lz);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace vr
