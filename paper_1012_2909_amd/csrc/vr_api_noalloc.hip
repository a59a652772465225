// vr_api_noalloc.hip -- vr_render without a caller workspace: the scratch the
// render needs lives in a fixed device array of this library.
//
// The only scratch vr_render uses outside save_for_backward is the per-pixel
// ray records of MIP in object order (64 bytes per pixel, written by the
// first kernel of that path before anything reads them).  Here they go into
// `scratch`, one copy per GPU, held until the process ends.  Its device
// address is resolved once per device, with that device current, by
// vr_noalloc_setup (called from vr_create); host code uses only that
// address, never the array's name.
#include <mutex>

#include "vr_ctx.h"

#define VR_NOALLOC_SCRATCH_BYTES (128LL << 20)   // 128 MiB: ray records of 2^21 pixels
#define VR_NOALLOC_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[VR_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[VR_NOALLOC_MAX_DEVICES];
static hipError_t g_scratch_err[VR_NOALLOC_MAX_DEVICES];

// Resolve this device's copy of the scratch array.  The caller has made
// `device` current.  Idempotent; the result (or the error) is kept.
void vr_noalloc_setup(int device) {
    if (device < 0 || device >= VR_NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    if (e == hipSuccess) g_scratch_ptr[device] = p;
}

extern "C" {

int64_t vr_render_noalloc_max_bytes(void) { return VR_NOALLOC_SCRATCH_BYTES; }

int vr_render_noalloc(vr_ctx *ctx, const vr_render_params *p, float *out_dev, void *stream) {
    if (!ctx || !p) return vr_fail(ctx, VR_EINVAL, "NULL argument");
    if (p->save_for_backward)
        return vr_fail(ctx, VR_EINVAL,
                       "vr_render_noalloc keeps no checkpoints: render with vr_render and a workspace "
                       "that outlives the call for save_for_backward");
    if (ctx->device < 0) return vr_fail(ctx, VR_EDEVICE, "host-only context");
    const int64_t need = vr_render_workspace_bytes(ctx, p);
    if (need < 0) return (int)need;                 // state / argument error, message already set
    if (need > VR_NOALLOC_SCRATCH_BYTES)
        return vr_fail(ctx, VR_ENOMEM,
                       "this render needs %lld bytes of scratch; the fixed scratch holds %lld "
                       "(object-order MIP takes 64 bytes per pixel): use vr_render with a workspace",
                       (long long)need, (long long)VR_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if (need > 0) {
        if (ctx->device >= VR_NOALLOC_MAX_DEVICES) return vr_fail(ctx, VR_EUNSUPPORTED, "device id too large");
        {
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            ws = g_scratch_ptr[ctx->device];
        }
        if (!ws)
            return vr_fail(ctx, VR_EDEVICE, "scratch address of device %d unresolved (%s)", ctx->device,
                           hipGetErrorString(g_scratch_err[ctx->device]));
    }
    return vr_render(ctx, p, out_dev, ws, need, stream);
}

}  // extern "C"
