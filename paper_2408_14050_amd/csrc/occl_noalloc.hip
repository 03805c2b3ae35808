// occl_noalloc.hip -- occl_detect_noalloc: the exact path of occl_detect for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The frame's workspace -- candidate lists, segment and completion counters,
// the class-major prefix and the partials of D's statistics (automatic scan
// lengths) -- lives in `scratch`, a file-scope device array of
// OCCL_NOALLOC_SCRATCH_BYTES that every device the library runs on holds
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in): occl_init resolves the
// array's address on its device once, with that device current
// (scratch_resolve below), and every later use goes through that pointer.
// The kernels are the ones occl_detect launches; they take the workspace
// pointers as arguments as they take the context's own buffers there.
//
// Every call on one device shares that device's array, and the array keeps
// the last call's contents: the counters that must start at zero are
// cleared by a fill kernel at the start of every call, and calls that
// overlap on one device (several streams or contexts) race.
#include <algorithm>
#include <cstdio>
#include <mutex>
#include <vector>

#include "occl_ctx.h"
#include "occl_internal.h"

using namespace occl;

namespace {

constexpr size_t kScratchBytes = (size_t)OCCL_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Layout: counters | prefix | statistics partials | candidate lists.
constexpr size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
constexpr size_t kOffCounts = 0;
constexpr size_t kOffPrefix = align256(kOffCounts + kCountsBytes);
constexpr size_t kOffStats = align256(kOffPrefix + kPrefixInts * sizeof(int32_t));
constexpr size_t kOffLists = align256(kOffStats + (3 + 3 * (size_t)kStatsBlocks) * sizeof(uint32_t));
static_assert(kOffLists < kScratchBytes, "the fixed part of the scratch layout must fit");

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device: the array's address there

}  // namespace

occl_status occl::scratch_resolve(int device, void** out) {
    if (device < 0 || !out) return OCCL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return OCCL_ERR_HIP;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return OCCL_OK;
}

extern "C" occl_status occl_detect_noalloc(occl_ctx* ctx, const float* D, int32_t H, int32_t W,
                                           int32_t n_views, const double* angles_deg,
                                           const float* ratios, const occl_params* params,
                                           uint8_t* M) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    occl_status s = ctx->check_params(params, n_views, angles_deg, ratios);
    if (s != OCCL_OK) return s;
    if (params->flags & OCCL_FLAG_USE_CNN)
        return ctx->fail(OCCL_ERR_UNSUPPORTED, "occl_detect_noalloc: the learned proposal needs the "
                                               "context's network workspace");
    if (H < 0 || W < 0) return ctx->fail(OCCL_ERR_INVALID_ARG, "negative size");
    if ((size_t)H * W == 0 || n_views == 0) return OCCL_OK;
    if (!D || !M) return ctx->fail(OCCL_ERR_INVALID_ARG, "D or M is NULL");
    if (H > 65535 || W > 65535) return ctx->fail(OCCL_ERR_UNSUPPORTED, "frame too large");
    if (!ctx->scratch) return ctx->fail(OCCL_ERR_STATE, "no scratch address for this device");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipSetDevice");
    uint8_t* base = static_cast<uint8_t*>(ctx->scratch);
    ViewTable vt{};
    int Ls[OCCL_MAX_VIEWS];
    // automatic scan lengths read D's statistics through the scratch's
    // partials (and synchronise, as in occl_detect)
    s = ctx->resolve_views(D, H, W, n_views, angles_deg, ratios, params, nullptr, &vt, Ls,
                           base + kOffStats);
    if (s != OCCL_OK) return s;
    const Thresholds th = make_thresholds(params);
    // the launch shape occl_detect would take for this frame, and the lists
    // it needs
    int maxcls = 0;
    for (int v = 0; v < n_views; ++v) maxcls = std::max(maxcls, scan_class(Ls[v] / 2, th.thin));
    TuneConfig tc = ctx->config_for(tune_key(false, (size_t)H * W, n_views, maxcls));
    if (tc.edge_rows < 1) tc.edge_rows = ctx->tune_default.edge_rows;
    FrameDesc f;
    describe_frame(&f, D, M, H, W, n_views, Ls, tc.edge_rows, th.thin);
    const size_t need = kOffLists + list_entries(f, n_views) * sizeof(uint32_t);
    if (need > kScratchBytes) {
        char msg[256];
        std::snprintf(msg, sizeof msg,
                      "occl_detect_noalloc: a %d x %d frame with %d views needs %zu bytes of scratch; "
                      "the static scratch holds %zu",
                      (int)W, (int)H, (int)n_views, need, kScratchBytes);
        return ctx->fail(OCCL_ERR_UNSUPPORTED, msg);
    }
    FrameWorkspace ws{reinterpret_cast<uint32_t*>(base + kOffLists),
                      reinterpret_cast<int32_t*>(base + kOffCounts),
                      reinterpret_cast<int32_t*>(base + kOffPrefix)};
    e = launch_fill_u32(ctx->stream, reinterpret_cast<uint32_t*>(ws.counts), (long long)kCountsInts);
    if (e != hipSuccess) return ctx->hip_fail(e, "clear scratch counters");
    s = ctx->enqueue_frame(D, H, W, n_views, Ls, vt, th, M, &tc, &ws);
    if (s != OCCL_OK) return s;
    if (params->flags & OCCL_FLAG_SYNC) {
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
    }
    return OCCL_OK;
}
