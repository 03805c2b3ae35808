// occl_batch.hip -- occl_detect_batched: many frames of uneven size.
#include <vector>

#include "occl_ctx.h"
#include "occl_internal.h"

using namespace occl;

extern "C" occl_status occl_detect_batched(occl_ctx* ctx, int32_t n_frames, const occl_frame* frames,
                                           int32_t n_views, const double* angles_deg,
                                           const float* ratios, const occl_params* params) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (n_frames < 0 || (n_frames > 0 && !frames)) return ctx->fail(OCCL_ERR_INVALID_ARG, "frames");
    occl_status s = ctx->check_params(params, n_views, angles_deg, ratios);
    if (s != OCCL_OK) return s;
    if (params->flags & OCCL_FLAG_USE_CNN) return ctx->fail(OCCL_ERR_UNSUPPORTED, "USE_CNN in a batch");
    for (int f = 0; f < n_frames; ++f) {
        const occl_frame& fr = frames[f];
        if (fr.H < 0 || fr.W < 0) return ctx->fail(OCCL_ERR_INVALID_ARG, "negative frame size");
        if ((size_t)fr.H * fr.W > 0 && n_views > 0 && (!fr.D || !fr.M))
            return ctx->fail(OCCL_ERR_INVALID_ARG, "frame D or M is NULL");
        if (fr.scan_len_per_view)
            for (int v = 0; v < n_views; ++v)
                if (fr.scan_len_per_view[v] < 1) return ctx->fail(OCCL_ERR_INVALID_ARG, "frame L < 1");
    }
    if (n_frames == 0 || n_views == 0) return OCCL_OK;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipSetDevice");
    const Thresholds th = make_thresholds(params);
    for (int f = 0; f < n_frames; ++f) {
        const occl_frame& fr = frames[f];
        if ((size_t)fr.H * fr.W == 0) continue;
        ViewTable vt{};
        int Ls[OCCL_MAX_VIEWS];
        s = ctx->resolve_views(fr.D, fr.H, fr.W, n_views, angles_deg, ratios, params,
                               fr.scan_len_per_view, &vt, Ls);
        if (s != OCCL_OK) return s;
        s = ctx->enqueue_frame(fr.D, fr.H, fr.W, n_views, vt, th, fr.M);
        if (s != OCCL_OK) return s;
    }
    if (params->flags & OCCL_FLAG_SYNC) {
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
    }
    return OCCL_OK;
}

occl_status occl_ctx::enqueue_frame_cnn(const float*, int, int, int, const ViewTable&,
                                        const Thresholds&, const occl_params*, uint8_t*) {
    return fail(OCCL_ERR_NO_MODEL, "learned tile proposal not loaded");
}
