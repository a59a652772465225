// k_pyramid.hip -- the display pyramid of a rendered frame (section 3: the
// high-resolution render is stored as a TIFF and converted to a pyramidal
// tiled TIFF for the tiled display's image server).
//
// Level 0 is the premultiplied RGBA float image quantised to 8 bits per
// channel; level l+1 averages 2x2 pixels of level l.  Everything after the
// quantisation is integer arithmetic, and the quantisation itself is exact
// (FP64 holds clamp(v)*255 + 1/2 of an FP32 v exactly), so the pyramid is a
// pure function of the image.  HBM-bound: one read of the float image and
// writes of 4/3 of level 0; a level is read back once for the next.
#include "vr_internal.h"

namespace vr {

__device__ __forceinline__ uint32_t quant8(float v) {
    // NaN -> 0; round half up of clamp(v, 0, 1) * 255, exact in FP64
    const float c = v > 0.0f ? fminf(v, 1.0f) : 0.0f;
    return (uint32_t)floor((double)c * 255.0 + 0.5);
}

// Level 0: one pixel per thread, a 16-byte load and a 4-byte store.
__global__ __launch_bounds__(256) void k_quant8(const float4 *src, uint32_t *dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 v = src[i];
    dst[i] = quant8(v.x) | (quant8(v.y) << 8) | (quant8(v.z) << 16) | (quant8(v.w) << 24);
}

// Level l+1 from level l (w x h): pixel (x, y) is the rounded mean of the
// n <= 4 pixels (2x + a, 2y + b) that exist, per channel (sum + n/2) / n.
__global__ __launch_bounds__(256) void k_down2(const uint32_t *src, int32_t w, int32_t h, uint32_t *dst, int32_t w2,
                                               int32_t h2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)w2 * h2) return;
    const int32_t x = (int32_t)(i % w2), y = (int32_t)(i / w2);
    const int32_t x0 = 2 * x, y0 = 2 * y;
    const bool hx = x0 + 1 < w, hy = y0 + 1 < h;
    const uint32_t n = (1u + hx) * (1u + hy);
    const uint32_t p00 = src[(int64_t)y0 * w + x0];
    const uint32_t p10 = hx ? src[(int64_t)y0 * w + x0 + 1] : 0u;
    const uint32_t p01 = hy ? src[(int64_t)(y0 + 1) * w + x0] : 0u;
    const uint32_t p11 = (hx && hy) ? src[(int64_t)(y0 + 1) * w + x0 + 1] : 0u;
    uint32_t out = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t s = ((p00 >> (8 * c)) & 255u) + ((p10 >> (8 * c)) & 255u) + ((p01 >> (8 * c)) & 255u) +
                           ((p11 >> (8 * c)) & 255u);
        out |= ((s + n / 2u) / n) << (8 * c);
    }
    dst[i] = out;
}

hipError_t launch_pyramid(const float *src, int32_t w, int32_t h, int32_t levels, uint8_t *dst, hipStream_t s) {
    if ((int64_t)w * h == 0) return hipSuccess;
    int64_t n = (int64_t)w * h;
    hipLaunchKernelGGL(k_quant8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float4 *)src,
                       (uint32_t *)dst, n);
    hipError_t e = hipGetLastError();
    uint32_t *cur = (uint32_t *)dst;
    for (int32_t l = 1; l < levels && e == hipSuccess; ++l) {
        const int32_t w2 = (w + 1) / 2, h2 = (h + 1) / 2;
        uint32_t *nxt = cur + (int64_t)w * h;
        const int64_t m = (int64_t)w2 * h2;
        hipLaunchKernelGGL(k_down2, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, cur, w, h, nxt, w2, h2);
        e = hipGetLastError();
        cur = nxt;
        w = w2;
        h = h2;
    }
    return e;
}

}  // namespace vr
