// vr_api_depth.hip -- C ABI of the depth pass and the catalogue overlay
// (include/vr.h): argument and state checks, then one launch each.
#include <cmath>

#include "vr_ctx.h"

using namespace vr;

extern "C" {

int vr_render_depth(vr_ctx *ctx, const vr_render_params *p, float level, float *depth_dev, void *stream) {
    int rc = vr_need_state(ctx, p && p->mode == VR_COMPOSITE);
    if (rc != VR_OK) return rc;
    if ((rc = vr_check_params(ctx, p)) != VR_OK) return rc;
    if (!depth_dev) return vr_fail(ctx, VR_EINVAL, "depth output is NULL");
    if (p->mode == VR_COMPOSITE && !(level > 0.0f && level <= 1.0f))
        return vr_fail(ctx, VR_EINVAL, "opacity level %g not in (0, 1]", (double)level);
    if (!ctx->vol.single) return vr_fail(ctx, VR_EUNSUPPORTED, "depth needs a one-brick layout");
    MarchArgs a = vr_march_args(ctx, p, ctx->camd);
    return vr_dev_check(ctx, launch_depth(a, p->mode, p->filter, level, depth_dev, (hipStream_t)stream), "depth");
}

int vr_overlay_boxes(vr_ctx *ctx, const vr_box *boxes_dev, int32_t n, float half_width, const float *depth_dev,
                     float *image_dev, void *stream) {
    if (!ctx) return vr_fail(nullptr, VR_EINVAL, "context is NULL");
    if (!ctx->has_camera) return vr_fail(ctx, VR_ESTATE, "vr_set_camera first");
    if (n < 0) return vr_fail(ctx, VR_EINVAL, "box count %d < 0", n);
    if (n > 0 && !boxes_dev) return vr_fail(ctx, VR_EINVAL, "boxes are NULL");
    if (!image_dev) return vr_fail(ctx, VR_EINVAL, "image is NULL");
    if (!(half_width > 0.0f && half_width <= 64.0f))
        return vr_fail(ctx, VR_EINVAL, "half width %g not in (0, 64]", (double)half_width);
    if (ctx->device < 0) return vr_fail(ctx, VR_EDEVICE, "host-only context");
    return vr_dev_check(ctx, launch_overlay(ctx->camd, boxes_dev, n, (double)half_width, 1e-3, depth_dev, image_dev,
                                            (hipStream_t)stream),
                        "overlay");
}

}  // extern "C"
