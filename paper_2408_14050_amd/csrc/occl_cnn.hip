// occl_cnn.hip -- host side of the learned tile proposal: model state,
// forward / backward / Adam on the k_cnn.hip kernels, and the C ABI.
#include <cmath>
#include <cstring>
#include <vector>

#include "occl_cnn.h"
#include "occl_ctx.h"

using namespace occl;

namespace {

struct Layer {
    int cin, cout, stride;
    bool relu;
};
const Layer kLayers[kCnnLayers] = {{8, 32, 2, true},  {32, 32, 2, true}, {32, 32, 2, true},
                                   {32, 32, 2, true}, {32, 32, 1, true}, {32, 1, 1, false}};

size_t off_w(int l) {
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += (size_t)kLayers[i].cout * 9 * kLayers[i].cin + kLayers[i].cout;
    return o;
}

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

size_t occl::cnn_num_params() { return off_w(kCnnLayers); }

void occl::cnn_dims(int H, int W, int* Hs, int* Ws) {
    Hs[0] = H;
    Ws[0] = W;
    for (int l = 0; l < kCnnLayers; ++l) {
        Hs[l + 1] = (Hs[l] + kLayers[l].stride - 1) / kLayers[l].stride;
        Ws[l + 1] = (Ws[l] + kLayers[l].stride - 1) / kLayers[l].stride;
    }
}

occl_status occl_ctx::cnn_buffers(float** theta, uint16_t** wbf) {
    const size_t P = cnn_num_params();
    void *a, *b;
    occl_status s = ensure("cnn_theta", P * sizeof(float), &a);
    if (s == OCCL_OK) s = ensure("cnn_wbf", P * sizeof(uint16_t), &b);
    if (s != OCCL_OK) return s;
    *theta = (float*)a;
    *wbf = (uint16_t*)b;
    return OCCL_OK;
}

// Forward pass of N samples of H x W x 8 (bf16 NHWC); logits to Z [N][Ht][Wt].
// Activations stay in the context workspace for a following backward pass.
// Layers first..5 on the input `in` of layer `first` (N samples of an H x W
// network input); logits to Z.  Activations stay in the context workspace.
occl_status occl_ctx::cnn_layers(int first, const uint16_t* in, int N, int H, int W, float* Z) {
    float* theta;
    uint16_t* wbf;
    occl_status s = cnn_buffers(&theta, &wbf);
    if (s != OCCL_OK) return s;
    int Hs[kCnnLayers + 1], Ws[kCnnLayers + 1];
    cnn_dims(H, W, Hs, Ws);
    for (int l = first; l < kCnnLayers - 1; ++l) {
        char name[16];
        std::snprintf(name, sizeof(name), "cnn_a%d", l);
        void* out;
        s = ensure(name, (size_t)N * Hs[l + 1] * Ws[l + 1] * 32 * sizeof(uint16_t), &out);
        if (s != OCCL_OK) return s;
        const size_t o = off_w(l);
        hipError_t e = cnn_conv_fwd(stream, kLayers[l].cin, kLayers[l].stride, in, wbf + o,
                                    theta + o + (size_t)32 * 9 * kLayers[l].cin, (uint16_t*)out, N,
                                    Hs[l], Ws[l], Hs[l + 1], Ws[l + 1], n_cu);
        if (e != hipSuccess) return hip_fail(e, "cnn conv fwd");
        cnn_act[l] = (uint16_t*)out;
        in = (const uint16_t*)out;
    }
    const size_t o5 = off_w(kCnnLayers - 1);
    hipError_t e = cnn_conv_last(stream, in, wbf + o5, theta + o5 + 9 * 32, Z, N, Hs[5], Ws[5]);
    if (e != hipSuccess) return hip_fail(e, "cnn conv last");
    cnn_fwd_n = N;
    cnn_fwd_h = H;
    cnn_fwd_w = W;
    return OCCL_OK;
}

// Forward pass of N samples of H x W x 8 (bf16 NHWC); logits to Z [N][Ht][Wt].
occl_status occl_ctx::cnn_forward(const uint16_t* X, int N, int H, int W, float* Z) {
    return cnn_layers(0, X, N, H, W, Z);
}

// The proposal of a frame: every view's logits straight from D (layer 0
// reads D through the per-frame base planes; bit-identical to packing every
// view and running cnn_forward).
occl_status occl_ctx::cnn_forward_frame(const float* D, int H, int W, int n_views, const ViewTable& vt,
                                        const int* Ls, float* Z) {
    float* theta;
    uint16_t* wbf;
    occl_status s = cnn_buffers(&theta, &wbf);
    if (s != OCCL_OK) return s;
    int Hs[kCnnLayers + 1], Ws[kCnnLayers + 1];
    cnn_dims(H, W, Hs, Ws);
    void *G, *a1;
    s = ensure("cnn_g", (size_t)H * W * sizeof(uint4), &G);
    if (s == OCCL_OK) s = ensure("cnn_a1", (size_t)n_views * Hs[2] * Ws[2] * 32 * sizeof(uint16_t), &a1);
    if (s != OCCL_OK) return s;
    const size_t o1 = off_w(1);
    hipError_t e = cnn_first_layers_fused(stream, D, H, W, n_views, vt, Ls, (uint4*)G, wbf,
                                          theta + (size_t)32 * 9 * kCnnInCh, wbf + o1,
                                          theta + o1 + (size_t)32 * 9 * 32, (uint16_t*)a1, Hs[1], Ws[1],
                                          Hs[2], Ws[2], n_cu);
    if (e != hipSuccess) return hip_fail(e, "cnn first layers");
    cnn_act[0] = nullptr;  // layer 0's output never leaves LDS
    cnn_act[1] = (const uint16_t*)a1;
    return cnn_layers(2, (const uint16_t*)a1, n_views, H, W, Z);
}

// Loss (mean soft BCE against T) and the gradient of every parameter into
// the "cnn_grad" workspace.
occl_status occl_ctx::cnn_backward(const uint16_t* X, int N, int H, int W, const float* T,
                                   double* loss) {
    int Hs[kCnnLayers + 1], Ws[kCnnLayers + 1];
    cnn_dims(H, W, Hs, Ws);
    const size_t P = cnn_num_params();
    const long ntile = (long)N * Hs[5] * Ws[5];
    void *z, *dz, *grad, *wt, *part, *bce, *g0, *g1;
    const size_t gmax = (size_t)N * Hs[1] * Ws[1] * 32;
    size_t pmax = 0;
    for (int l = 0; l < kCnnLayers - 1; ++l)
        pmax = std::max(pmax, cnn_wgrad_partial_floats((long)N * Hs[l + 1] * Ws[l + 1], kLayers[l].cin));
    pmax = std::max(pmax, cnn_last_partial_floats(ntile));
    const int nb = 256;
    occl_status s = ensure("cnn_z", ntile * sizeof(float), &z);
    if (s == OCCL_OK) s = ensure("cnn_dz", ntile * sizeof(float), &dz);
    if (s == OCCL_OK) s = ensure("cnn_grad", P * sizeof(float), &grad);
    if (s == OCCL_OK) s = ensure("cnn_wt", 9 * 32 * 32 * sizeof(uint16_t), &wt);
    if (s == OCCL_OK) s = ensure("cnn_part", pmax * sizeof(float), &part);
    if (s == OCCL_OK) s = ensure("cnn_bce", nb * sizeof(double), &bce);
    if (s == OCCL_OK) s = ensure("cnn_g0", gmax * sizeof(uint16_t), &g0);
    if (s == OCCL_OK) s = ensure("cnn_g1", gmax * sizeof(uint16_t), &g1);
    if (s != OCCL_OK) return s;
    s = cnn_forward(X, N, H, W, (float*)z);
    if (s != OCCL_OK) return s;
    float* theta;
    uint16_t* wbf;
    cnn_buffers(&theta, &wbf);
    hipError_t e = cnn_bce(stream, (const float*)z, T, (float*)dz, (double*)bce, ntile, nb);
    if (e != hipSuccess) return hip_fail(e, "cnn bce");
    const size_t o5 = off_w(5);
    e = cnn_last_backward(stream, (const float*)dz, cnn_act[4], wbf + o5, (uint16_t*)g0, (float*)part,
                          (float*)grad + o5, N, Hs[5], Ws[5]);
    if (e != hipSuccess) return hip_fail(e, "cnn last backward");
    uint16_t* gin = (uint16_t*)g0;   // gradient of the current layer's output
    uint16_t* gout = (uint16_t*)g1;  // gradient of its input
    for (int l = kCnnLayers - 2; l >= 0; --l) {
        const uint16_t* Xl = l == 0 ? X : cnn_act[l - 1];
        const size_t o = off_w(l);
        e = cnn_layer_backward(stream, kLayers[l].cin, kLayers[l].stride, gin, cnn_act[l], Xl, wbf + o,
                               (uint16_t*)wt, l == 0 ? nullptr : gout, (float*)part, (float*)grad + o, N,
                               Hs[l], Ws[l], Hs[l + 1], Ws[l + 1]);
        if (e != hipSuccess) return hip_fail(e, "cnn layer backward");
        std::swap(gin, gout);
    }
    if (loss) {
        std::vector<double> h(nb);
        e = hipMemcpyAsync(h.data(), bce, nb * sizeof(double), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "cnn loss readback");
        double t = 0.0;
        for (double x : h) t += x;
        *loss = t / (double)ntile;
    }
    return OCCL_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace {
occl_status check_ctx_model(occl_ctx* ctx) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (!ctx->cnn_loaded) return ctx->fail(OCCL_ERR_NO_MODEL, "no CNN weights (occl_cnn_init / set_state)");
    return OCCL_OK;
}

occl_status check_xdims(occl_ctx* ctx, const void* X, int N, int H, int W) {
    if (!X || N < 1 || H < 1 || W < 1 || (long)N * H * W > (1l << 31))
        return ctx->fail(OCCL_ERR_INVALID_ARG, "CNN input shape");
    return OCCL_OK;
}
}  // namespace

extern "C" size_t occl_cnn_num_params(void) { return cnn_num_params(); }

extern "C" occl_status occl_cnn_init(occl_ctx* ctx, uint64_t seed) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    const size_t P = cnn_num_params();
    std::vector<float> th(P, 0.0f);
    uint64_t st = seed;
    for (int l = 0; l < kCnnLayers; ++l) {
        const size_t o = off_w(l);
        const size_t nw = (size_t)kLayers[l].cout * 9 * kLayers[l].cin;
        const double a = std::sqrt(6.0 / (9.0 * kLayers[l].cin));  // He-uniform
        for (size_t i = 0; i < nw; ++i) {
            const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
            th[o + i] = (float)((2.0 * u - 1.0) * a);
        }
    }
    std::vector<float> zeros(P, 0.0f);
    return occl_cnn_set_state(ctx, th.data(), zeros.data(), zeros.data(), 0, P);
}

extern "C" occl_status occl_cnn_set_state(occl_ctx* ctx, const float* theta, const float* m,
                                          const float* v, int64_t step, size_t n) {
    if (!ctx || !theta || n != cnn_num_params() || step < 0) return OCCL_ERR_INVALID_ARG;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(theta[i]) || (m && !std::isfinite(m[i])) || (v && !(v[i] >= 0.0f)))
            return ctx->fail(OCCL_ERR_INVALID_ARG, "non-finite model state");
    (void)hipSetDevice(ctx->device);
    float* dth;
    uint16_t* wbf;
    occl_status s = ctx->cnn_buffers(&dth, &wbf);
    void *dm, *dv;
    if (s == OCCL_OK) s = ctx->ensure("cnn_m", n * sizeof(float), &dm);
    if (s == OCCL_OK) s = ctx->ensure("cnn_v", n * sizeof(float), &dv);
    if (s != OCCL_OK) return s;
    hipError_t e = hipMemcpy(dth, theta, n * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = m ? hipMemcpy(dm, m, n * sizeof(float), hipMemcpyHostToDevice) : hipMemset(dm, 0, n * sizeof(float));
    if (e == hipSuccess)
        e = v ? hipMemcpy(dv, v, n * sizeof(float), hipMemcpyHostToDevice) : hipMemset(dv, 0, n * sizeof(float));
    if (e == hipSuccess) e = cnn_to_bf16(ctx->stream, dth, wbf, (int)n);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return ctx->hip_fail(e, "cnn set state");
    ctx->cnn_step = step;
    ctx->cnn_loaded = true;
    return OCCL_OK;
}

extern "C" occl_status occl_cnn_get_state(occl_ctx* ctx, float* theta, float* m, float* v,
                                          int64_t* step, size_t n) {
    occl_status s = check_ctx_model(ctx);
    if (s != OCCL_OK) return s;
    if (n != cnn_num_params()) return ctx->fail(OCCL_ERR_INVALID_ARG, "parameter count");
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    auto get = [&](const char* name, float* dst) {
        if (!dst || e != hipSuccess) return;
        e = hipMemcpy(dst, ctx->bufs[name].ptr, n * sizeof(float), hipMemcpyDeviceToHost);
    };
    get("cnn_theta", theta);
    get("cnn_m", m);
    get("cnn_v", v);
    if (e != hipSuccess) return ctx->hip_fail(e, "cnn get state");
    if (step) *step = ctx->cnn_step;
    return OCCL_OK;
}

extern "C" occl_status occl_cnn_activation(occl_ctx* ctx, int32_t layer, uint16_t* dst, size_t n) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (layer < 0 || layer >= kCnnLayers - 1 || !dst) return ctx->fail(OCCL_ERR_INVALID_ARG, "layer / dst");
    if (ctx->cnn_fwd_n == 0) return ctx->fail(OCCL_ERR_STATE, "no forward pass yet");
    if (!ctx->cnn_act[layer])
        return ctx->fail(OCCL_ERR_STATE, "layer not kept by the last forward pass (fused proposal)");
    int Hs[kCnnLayers + 1], Ws[kCnnLayers + 1];
    cnn_dims(ctx->cnn_fwd_h, ctx->cnn_fwd_w, Hs, Ws);
    const size_t want = (size_t)ctx->cnn_fwd_n * Hs[layer + 1] * Ws[layer + 1] * 32;
    if (n != want) return ctx->fail(OCCL_ERR_INVALID_ARG, "element count of the activation");
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipMemcpyAsync(dst, ctx->cnn_act[layer], n * sizeof(uint16_t), hipMemcpyDeviceToDevice,
                                  ctx->stream);
    if (e != hipSuccess) return ctx->hip_fail(e, "activation copy");
    return OCCL_OK;
}

extern "C" occl_status occl_cnn_pack(occl_ctx* ctx, const float* D, int32_t H, int32_t W,
                                     int32_t n_views, const double* angles_deg, const float* ratios,
                                     const int32_t* scan_len, uint16_t* X) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (!D || !X || !scan_len || H < 1 || W < 1 || n_views < 1 || n_views > OCCL_MAX_VIEWS ||
        !angles_deg || !ratios)
        return ctx->fail(OCCL_ERR_INVALID_ARG, "pack arguments");
    ViewTable vt{};
    for (int v = 0; v < n_views; ++v) {
        if (scan_len[v] < 1 || !(ratios[v] > 0.0f) || !std::isfinite(angles_deg[v]))
            return ctx->fail(OCCL_ERR_INVALID_ARG, "pack view");
        occl_direction(angles_deg[v], &vt.c[v], &vt.s[v]);
        vt.r[v] = ratios[v];
    }
    (void)hipSetDevice(ctx->device);
    hipError_t e = cnn_pack(ctx->stream, D, H, W, n_views, vt, scan_len, X);
    if (e != hipSuccess) return ctx->hip_fail(e, "cnn pack");
    return OCCL_OK;
}

extern "C" occl_status occl_cnn_propose(occl_ctx* ctx, const float* D, int32_t H, int32_t W,
                                        int32_t n_views, const double* angles_deg, const float* ratios,
                                        const int32_t* scan_len, float* logits) {
    occl_status s = check_ctx_model(ctx);
    if (s != OCCL_OK) return s;
    if (!D || !logits || !scan_len || !angles_deg || !ratios || H < 1 || W < 1 || n_views < 1 ||
        n_views > OCCL_MAX_VIEWS || (long)H * W > (1l << 31))
        return ctx->fail(OCCL_ERR_INVALID_ARG, "propose arguments");
    ViewTable vt{};
    int Ls[OCCL_MAX_VIEWS];
    for (int v = 0; v < n_views; ++v) {
        if (scan_len[v] < 1 || !(ratios[v] > 0.0f) || !std::isfinite(ratios[v]) || !std::isfinite(angles_deg[v]))
            return ctx->fail(OCCL_ERR_INVALID_ARG, "propose view");
        occl_direction(angles_deg[v], &vt.c[v], &vt.s[v]);
        vt.r[v] = ratios[v];
        Ls[v] = scan_len[v];
    }
    (void)hipSetDevice(ctx->device);
    return ctx->cnn_forward_frame(D, H, W, n_views, vt, Ls, logits);
}

extern "C" occl_status occl_cnn_tile_targets(occl_ctx* ctx, const uint8_t* M, int32_t n, int32_t H,
                                             int32_t W, float* T) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (!M || !T || n < 1 || H < 1 || W < 1) return ctx->fail(OCCL_ERR_INVALID_ARG, "tile targets");
    (void)hipSetDevice(ctx->device);
    hipError_t e = cnn_tile_targets(ctx->stream, M, n, H, W, T);
    if (e != hipSuccess) return ctx->hip_fail(e, "tile targets");
    return OCCL_OK;
}

extern "C" occl_status occl_cnn_forward(occl_ctx* ctx, const uint16_t* X, int32_t N, int32_t H,
                                        int32_t W, float* logits) {
    occl_status s = check_ctx_model(ctx);
    if (s == OCCL_OK) s = check_xdims(ctx, X, N, H, W);
    if (s != OCCL_OK) return s;
    if (!logits) return ctx->fail(OCCL_ERR_INVALID_ARG, "logits");
    (void)hipSetDevice(ctx->device);
    return ctx->cnn_forward(X, N, H, W, logits);
}

extern "C" occl_status occl_cnn_backward(occl_ctx* ctx, const uint16_t* X, int32_t N, int32_t H,
                                         int32_t W, const float* T, double* loss, float* grad) {
    occl_status s = check_ctx_model(ctx);
    if (s == OCCL_OK) s = check_xdims(ctx, X, N, H, W);
    if (s != OCCL_OK) return s;
    if (!T) return ctx->fail(OCCL_ERR_INVALID_ARG, "targets");
    (void)hipSetDevice(ctx->device);
    s = ctx->cnn_backward(X, N, H, W, T, loss);
    if (s != OCCL_OK || !grad) return s;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpy(grad, ctx->bufs["cnn_grad"].ptr, cnn_num_params() * sizeof(float),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ctx->hip_fail(e, "grad readback");
    return OCCL_OK;
}

extern "C" occl_status occl_cnn_train_step(occl_ctx* ctx, const uint16_t* X, int32_t N, int32_t H,
                                           int32_t W, const float* T, float lr, double* loss) {
    occl_status s = check_ctx_model(ctx);
    if (s == OCCL_OK) s = check_xdims(ctx, X, N, H, W);
    if (s != OCCL_OK) return s;
    if (!T || !(lr > 0.0f) || !std::isfinite(lr)) return ctx->fail(OCCL_ERR_INVALID_ARG, "targets / lr");
    (void)hipSetDevice(ctx->device);
    s = ctx->cnn_backward(X, N, H, W, T, loss);
    if (s != OCCL_OK) return s;
    const double b1 = 0.9, b2 = 0.999;
    const int64_t t = ctx->cnn_step + 1;
    const double bc1 = 1.0 - std::pow(b1, (double)t);
    const double bc2 = 1.0 - std::pow(b2, (double)t);
    float* theta;
    uint16_t* wbf;
    ctx->cnn_buffers(&theta, &wbf);
    hipError_t e = cnn_adam(ctx->stream, theta, (const float*)ctx->bufs["cnn_grad"].ptr,
                            (float*)ctx->bufs["cnn_m"].ptr, (float*)ctx->bufs["cnn_v"].ptr, wbf,
                            (int)cnn_num_params(), lr, b1, b2, 1e-8, bc1, bc2);
    if (e != hipSuccess) return ctx->hip_fail(e, "adam");
    ctx->cnn_step = t;
    return OCCL_OK;
}

// ---------------------------------------------------------------------------
// routing + exact fallback, and the full learned path
// ---------------------------------------------------------------------------
namespace {
// logit of a probability bound, in double, rounded to fp32 (0 -> -inf, 1 -> +inf)
float logit_bound(float p) {
    if (!(p > 0.0f)) return -INFINITY;
    if (!(p < 1.0f)) return INFINITY;
    return (float)std::log((double)p / (1.0 - (double)p));
}
}  // namespace

occl_status occl_ctx::enqueue_routed(const float* D, int H, int W, int n_views, const int* Ls,
                                     const ViewTable& vt, const Thresholds& th, const occl_params* p,
                                     const float* logits, uint8_t* M, uint8_t* tile_state) {
    const int ty = (H + kTile - 1) / kTile, tx = (W + kTile - 1) / kTile;
    const size_t nt = (size_t)n_views * ty * tx;
    void* st = tile_state;
    occl_status s = OCCL_OK;
    if (!st) s = ensure("tile_state", nt, &st);
    if (s != OCCL_OK) return s;
    hipEvent_t ev = prof_begin(OCCL_STAGE_FALLBACK);
    hipError_t e = launch_route_state(stream, logits, nt, logit_bound(p->cnn_lo), logit_bound(p->cnn_hi),
                                      (uint8_t*)st);
    if (e != hipSuccess) return hip_fail(e, "route states");
    // The exact path over the whole frame, then the confident tiles' fill.
    // Confident tiles hold no candidates in practice (they are far from any
    // depth edge), so restricting the exact path to the uncertain tiles and
    // their reach saves nothing; the plain kernels are the fastest form.
    s = enqueue_frame(D, H, W, n_views, Ls, vt, th, M, nullptr);
    if (s != OCCL_OK) return s;
    e = launch_route_apply(stream, (const uint8_t*)st, n_views, H, W, ty, tx, M);
    if (e != hipSuccess) return hip_fail(e, "route fill");
    prof_end(OCCL_STAGE_FALLBACK, ev);
    return OCCL_OK;
}

occl_status occl_ctx::enqueue_frame_cnn(const float* D, int H, int W, int n_views, const int* Ls,
                                        const ViewTable& vt, const Thresholds& th, const occl_params* p,
                                        uint8_t* M) {
    const int ty = (H + kTile - 1) / kTile, tx = (W + kTile - 1) / kTile;
    void* Z;
    occl_status s = ensure("cnn_logits", (size_t)n_views * ty * tx * sizeof(float), &Z);
    if (s != OCCL_OK) return s;
    hipEvent_t ev = prof_begin(OCCL_STAGE_CNN);
    s = cnn_forward_frame(D, H, W, n_views, vt, Ls, (float*)Z);
    if (s != OCCL_OK) return s;
    prof_end(OCCL_STAGE_CNN, ev);
    return enqueue_routed(D, H, W, n_views, Ls, vt, th, p, (const float*)Z, M, nullptr);
}
