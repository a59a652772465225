// Entry points whose device paths are not built yet: they validate nothing
// and report VR_EUNSUPPORTED.
#include "vr_internal.h"

extern "C" {
int64_t vr_batch_workspace_bytes(const vr_ctx *, const vr_view *, int32_t) { return VR_EUNSUPPORTED; }
int vr_render_batch(vr_ctx *, const vr_render_params *, const vr_view *, int32_t, const float *, int32_t, int32_t,
                    float, float, void *, int64_t, int32_t, void *) {
    return VR_EUNSUPPORTED;
}
int vr_autotune(vr_ctx *, const vr_render_params *, float *, void *, int64_t, const char *, void *) {
    return VR_EUNSUPPORTED;
}
}
