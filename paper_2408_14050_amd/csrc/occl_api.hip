// occl_api.hip -- host side of the C ABI declared in include/occl.h.
//
// Validation, per-view constants (direction vectors, half scan lengths),
// workspace management and the launch sequence of one frame:
//   [optional D statistics -> host]  k_edges_candidates  k_scanlines<K> per K.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "occl_ctx.h"
#include "occl_internal.h"

using namespace occl;

// ---------------------------------------------------------------------------
// status strings / errors
// ---------------------------------------------------------------------------
extern "C" const char* occl_status_string(occl_status s) {
    switch (s) {
        case OCCL_OK: return "ok";
        case OCCL_ERR_INVALID_ARG: return "invalid argument";
        case OCCL_ERR_OUT_OF_MEMORY: return "out of memory";
        case OCCL_ERR_HIP: return "HIP runtime error";
        case OCCL_ERR_UNSUPPORTED: return "unsupported";
        case OCCL_ERR_NO_MODEL: return "no model loaded";
        case OCCL_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

extern "C" const char* occl_last_error(const occl_ctx* ctx) {
    return ctx ? ctx->last_error.c_str() : "null context";
}

occl_status occl_ctx::fail(occl_status s, const char* what) {
    last_error = std::string(occl_status_string(s)) + ": " + what;
    return s;
}

occl_status occl_ctx::hip_fail(hipError_t e, const char* where) {
    last_error = std::string("HIP error in ") + where + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? OCCL_ERR_OUT_OF_MEMORY : OCCL_ERR_HIP;
}

// ---------------------------------------------------------------------------
// direction vector of a baseline angle (degrees): reduce modulo 360, split
// into quadrant q and b in [0, 90); b == 0 is exact; otherwise the octant
// reference angle psi in (0, 45] is evaluated in double (psi * pi / 180 with
// pi / 180 formed as 3.14159265358979323846 / 180), rounded to fp32 and
// mapped back by the quadrant rotation.
// ---------------------------------------------------------------------------
namespace {
void direction_of(double angle, float* c, float* s) {
    double a = std::fmod(angle, 360.0);
    if (a < 0.0) a += 360.0;
    if (a >= 360.0) a = 0.0;
    int q = (int)std::floor(a / 90.0);
    q = q > 3 ? 3 : q;
    const double b = a - 90.0 * q;
    const double rad = 3.14159265358979323846 / 180.0;
    float u, w;  // (cos b, sin b) in fp32
    if (b == 0.0) {
        u = 1.0f;
        w = 0.0f;
    } else if (b <= 45.0) {
        u = (float)std::cos(b * rad);
        w = (float)std::sin(b * rad);
    } else {
        const double p = 90.0 - b;
        u = (float)std::sin(p * rad);
        w = (float)std::cos(p * rad);
    }
    const float cs[4][2] = {{u, w}, {-w, u}, {-u, -w}, {w, -u}};
    *c = cs[q][0];
    *s = cs[q][1];
}
}  // namespace

extern "C" occl_status occl_direction(double angle_deg, float* c, float* s) {
    if (!c || !s || !std::isfinite(angle_deg)) return OCCL_ERR_INVALID_ARG;
    direction_of(angle_deg, c, s);
    return OCCL_OK;
}

extern "C" void occl_params_default(occl_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(occl_params);
    p->edge_thr = 1.0f;
    p->disp_thr = 0.5f;
    p->dist_thr = 1.0f;
    p->neighbours = 1;
    p->scan_len = 0;
    p->scan_len_per_view = nullptr;
    p->flags = 0;
    p->cnn_lo = 0.05f;
    p->cnn_hi = 0.95f;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
occl_ctx::~occl_ctx() {
    (void)hipStreamSynchronize(stream);
    for (auto& p : ev_pairs) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto& g : graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
    if (table_event) (void)hipEventSynchronize(table_event);
    if (table_event) (void)hipEventDestroy(table_event);
    if (table_host) (void)hipHostFree(table_host);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& st : cap_extra)
        if (st) (void)hipStreamDestroy(st);
    if (cap_fork) (void)hipEventDestroy(cap_fork);
    for (auto& ev : cap_join)
        if (ev) (void)hipEventDestroy(ev);
    free_all();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void occl_ctx::free_all() {
    table_cached_dev = nullptr;
    for (auto& b : bufs) {
        if (b.second.ptr) (void)hipFree(b.second.ptr);
    }
    bufs.clear();
    if (host_stats) (void)hipHostFree(host_stats);
    host_stats = nullptr;
}

occl_status occl_ctx::ensure(const char* name, size_t bytes, void** out) {
    Buf& b = bufs[name];
    if (b.bytes >= bytes && b.ptr) {
        *out = b.ptr;
        return OCCL_OK;
    }
    if (workspace_cap && total_bytes() - b.bytes + bytes > workspace_cap)
        return fail(OCCL_ERR_OUT_OF_MEMORY, "workspace cap exceeded");
    if (b.ptr) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
        drop_graphs();
    }
    size_t alloc = bytes < 256 ? 256 : bytes;
    table_cached_dev = nullptr;  // a new buffer may reuse a freed one's address
    hipError_t e = hipMalloc(&b.ptr, alloc);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        (void)hipGetLastError();
        return hip_fail(e, "hipMalloc(workspace)");
    }
    b.bytes = alloc;
    *out = b.ptr;
    return OCCL_OK;
}

// Like ensure(), but a new allocation is cleared (synchronously) before use.
occl_status occl_ctx::ensure_zeroed(const char* name, size_t bytes, void** out) {
    const bool fresh = bufs.find(name) == bufs.end() || bufs[name].bytes < bytes;
    occl_status s = ensure(name, bytes, out);
    if (s != OCCL_OK || !fresh) return s;
    hipError_t e = hipMemset(*out, 0, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipMemset(workspace)");
    return OCCL_OK;
}

void occl_ctx::drop_graphs() {
    for (auto& g : graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
}

size_t occl_ctx::total_bytes() const {
    size_t t = 0;
    for (const auto& b : bufs) t += b.second.bytes;
    return t;
}

extern "C" occl_status occl_init(occl_ctx** out, int device, void* hip_stream,
                                 size_t max_pixels_hint, int32_t max_views_hint) {
    if (!out) return OCCL_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return OCCL_ERR_HIP;
    if (device < 0 || device >= ndev) return OCCL_ERR_INVALID_ARG;
    if (max_views_hint < 0 || max_views_hint > OCCL_MAX_VIEWS) return OCCL_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return OCCL_ERR_HIP;
    occl_ctx* ctx = new (std::nothrow) occl_ctx();
    if (!ctx) return OCCL_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    // NULL: the context creates and owns a stream of its own (default
    // priority; blocking, so it still orders itself with the device's null
    // stream), destroyed by occl_release.
    ctx->stream = (hipStream_t)hip_stream;
    ctx->own_stream = false;
    if (!ctx->stream) {
        if (hipStreamCreate(&ctx->stream) != hipSuccess) {
            (void)hipGetLastError();
            ctx->stream = nullptr;
            delete ctx;
            return OCCL_ERR_HIP;
        }
        ctx->own_stream = true;
    }
    if (hipHostMalloc((void**)&ctx->host_stats, 64, hipHostMallocDefault) != hipSuccess) {
        ctx->host_stats = nullptr;
        delete ctx;
        return OCCL_ERR_OUT_OF_MEMORY;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        cus = 256;
    ctx->n_cu = cus;
    // the address of this device's static scratch array (occl_detect_noalloc),
    // resolved once per device with the device current
    occl_status ss = scratch_resolve(device, &ctx->scratch);
    if (ss != OCCL_OK) {
        delete ctx;
        return ss;
    }
    void* p;
    occl_status s = ctx->ensure_zeroed("counts", kCountsBytes, &p);
    if (s == OCCL_OK && max_pixels_hint > 0 && max_views_hint > 0)
        s = ctx->ensure("lists", (max_pixels_hint + (size_t)kMaxCopies * kMaxEdgeRows * 4096) *
                                     max_views_hint * sizeof(uint32_t), &p);
    if (s != OCCL_OK) {
        delete ctx;
        return s;
    }
    *out = ctx;
    return OCCL_OK;
}

extern "C" occl_status occl_set_workspace_cap(occl_ctx* ctx, size_t bytes) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    ctx->workspace_cap = bytes;
    return OCCL_OK;
}

extern "C" occl_status occl_workspace_bytes(const occl_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return OCCL_ERR_INVALID_ARG;
    *bytes = ctx->total_bytes();
    return OCCL_OK;
}

extern "C" occl_status occl_release(occl_ctx* ctx) {
    if (!ctx) return OCCL_OK;
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    delete ctx;
    return e == hipSuccess ? OCCL_OK : OCCL_ERR_HIP;
}

extern "C" occl_status occl_sync(occl_ctx* ctx) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
    return OCCL_OK;
}

// ---------------------------------------------------------------------------
// validation + per-view constants
// ---------------------------------------------------------------------------
occl_status occl_ctx::check_params(const occl_params* p, int n_views, const double* angles,
                                   const float* ratios) {
    if (!p) return fail(OCCL_ERR_INVALID_ARG, "params is NULL");
    if (p->struct_size != sizeof(occl_params)) return fail(OCCL_ERR_INVALID_ARG, "params.struct_size");
    if (!std::isfinite(p->edge_thr) || !std::isfinite(p->disp_thr) || !std::isfinite(p->dist_thr))
        return fail(OCCL_ERR_INVALID_ARG, "non-finite threshold");
    if (p->neighbours < 1 || p->neighbours > OCCL_MAX_NEIGHBOURS)
        return fail(OCCL_ERR_INVALID_ARG, "neighbours out of range");
    if (p->scan_len < -1 && !p->scan_len_per_view) return fail(OCCL_ERR_INVALID_ARG, "scan_len < -1");
    if (n_views < 0 || n_views > OCCL_MAX_VIEWS) return fail(OCCL_ERR_INVALID_ARG, "n_views out of range");
    if (n_views > 0 && (!angles || !ratios)) return fail(OCCL_ERR_INVALID_ARG, "angles/ratios NULL");
    for (int v = 0; v < n_views; ++v) {
        if (!std::isfinite(angles[v])) return fail(OCCL_ERR_INVALID_ARG, "non-finite angle");
        if (!std::isfinite(ratios[v]) || !(ratios[v] > 0.0f))
            return fail(OCCL_ERR_INVALID_ARG, "ratio must be finite and > 0");
        if (p->scan_len_per_view && p->scan_len_per_view[v] < 1)
            return fail(OCCL_ERR_INVALID_ARG, "scan_len_per_view[v] < 1");
    }
    if ((p->flags & OCCL_FLAG_USE_CNN) && !(p->cnn_lo <= p->cnn_hi))
        return fail(OCCL_ERR_INVALID_ARG, "cnn band");
    return OCCL_OK;
}

// Reads min / max / non-finite count of D back to the host (synchronises).
occl_status occl_ctx::d_stats(const float* D, size_t n, float* mn, float* mx, uint32_t* bad,
                              void* stats_ws) {
    void* dev = stats_ws;
    if (!dev) {
        occl_status s = ensure("stats", (3 + 3 * (size_t)kStatsBlocks) * sizeof(uint32_t), &dev);
        if (s != OCCL_OK) return s;
    }
    hipError_t e = launch_scan_stats(stream, D, n, (uint32_t*)dev);
    if (e != hipSuccess) return hip_fail(e, "scan_stats");
    e = hipMemcpyAsync(host_stats, dev, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(stats)");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(stats)");
    auto unord = [](uint32_t o) {
        uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    };
    *mn = unord(host_stats[0]);
    *mx = unord(host_stats[1]);
    *bad = host_stats[2];
    return OCCL_OK;
}

// Per-view L from the params (possibly from D's statistics); returns the
// table of direction vectors and half lengths.
occl_status occl_ctx::resolve_views(const float* D, int H, int W, int n_views,
                                    const double* angles, const float* ratios,
                                    const occl_params* p, const int32_t* frame_L, ViewTable* vt,
                                    int* Ls, void* stats_ws) {
    bool need_stats = false;
    for (int v = 0; v < n_views; ++v) {
        int L = frame_L ? frame_L[v] : (p->scan_len_per_view ? p->scan_len_per_view[v] : p->scan_len);
        if (L <= 0) need_stats = true;
        Ls[v] = L;
    }
    const bool validate = (p->flags & OCCL_FLAG_VALIDATE_INPUT) != 0;
    if (need_stats || validate) {
        float mn, mx;
        uint32_t bad;
        occl_status s = d_stats(D, (size_t)H * W, &mn, &mx, &bad, stats_ws);
        if (s != OCCL_OK) return s;
        if (bad) return fail(OCCL_ERR_INVALID_ARG, "D holds non-finite values");
        for (int v = 0; v < n_views; ++v) {
            if (Ls[v] > 0) continue;
            const float r = ratios[v];
            double Lr;
            if (Ls[v] == 0) {
                volatile float prod = mx * r;  // fp32 product
                Lr = std::ceil((double)prod) + 2.0;
            } else {
                volatile float span = mx - mn;
                volatile float t = span * r;
                volatile float q = t * 2.0f;
                Lr = std::ceil((double)q);
            }
            if (Lr < 1.0) Lr = 1.0;
            if (Lr > 1e9) Lr = 1e9;
            Ls[v] = (int)Lr;
        }
    }
    for (int v = 0; v < n_views; ++v) {
        if (Ls[v] < 1) return fail(OCCL_ERR_INVALID_ARG, "scan length < 1");
        if (Ls[v] > OCCL_MAX_SCAN_LEN) return fail(OCCL_ERR_UNSUPPORTED, "scan length > 1023");
        if ((p->flags & OCCL_FLAG_THIN) && Ls[v] > OCCL_THIN_MAX_SCAN_LEN)
            return fail(OCCL_ERR_UNSUPPORTED, "scan length > 683 with candidate thinning");
        direction_of(angles[v], &vt->c[v], &vt->s[v]);
        vt->r[v] = ratios[v];
    }
    return OCCL_OK;
}

// ---------------------------------------------------------------------------
// stage profiling
// ---------------------------------------------------------------------------
hipEvent_t occl_ctx::take_event() {
    if (!ev_pool.empty()) {
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipEvent_t occl_ctx::prof_begin(int stage) {
    (void)stage;
    if (!profiling) return nullptr;
    if (ev_pairs.size() > 8192) (void)prof_resolve();
    hipEvent_t a = take_event();
    if (a && hipEventRecord(a, stream) != hipSuccess) {
        ev_pool.push_back(a);
        return nullptr;
    }
    return a;
}

void occl_ctx::prof_end(int stage, hipEvent_t a) {
    if (!profiling || !a) return;
    hipEvent_t b = take_event();
    if (!b || hipEventRecord(b, stream) != hipSuccess) {
        ev_pool.push_back(a);
        if (b) ev_pool.push_back(b);
        return;
    }
    ev_pairs.push_back(EvPair{stage, a, b});
}

occl_status occl_ctx::prof_resolve() {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(profile)");
    for (auto& p : ev_pairs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            prof_ms[p.stage] += ms;
            prof_n[p.stage] += 1;
        }
        ev_pool.push_back(p.a);
        ev_pool.push_back(p.b);
    }
    ev_pairs.clear();
    return OCCL_OK;
}

extern "C" occl_status occl_profile_enable(occl_ctx* ctx, int32_t enable) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    occl_status s = ctx->prof_resolve();
    if (s != OCCL_OK) return s;
    for (int i = 0; i < OCCL_N_STAGES; ++i) {
        ctx->prof_ms[i] = 0.0;
        ctx->prof_n[i] = 0;
    }
    ctx->profiling = enable != 0;
    return OCCL_OK;
}

extern "C" occl_status occl_profile_read(occl_ctx* ctx, double* ms, int64_t* launches) {
    if (!ctx || !ms || !launches) return OCCL_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    occl_status s = ctx->prof_resolve();
    if (s != OCCL_OK) return s;
    for (int i = 0; i < OCCL_N_STAGES; ++i) {
        ms[i] = ctx->prof_ms[i];
        launches[i] = ctx->prof_n[i];
    }
    return OCCL_OK;
}

// Enqueues the exact path of one frame (launch shape: cfg, else the tuned or
// default shape for this frame).
occl_status occl_ctx::enqueue_frame(const float* D, int H, int W, int n_views, const int* Ls,
                                    const ViewTable& vt, const Thresholds& th, uint8_t* M,
                                    const TuneConfig* cfg, const FrameWorkspace* ws) {
    int maxcls = 0;
    for (int v = 0; v < n_views; ++v) maxcls = std::max(maxcls, scan_class(Ls[v] / 2, th.thin));
    TuneConfig tc = cfg ? *cfg : config_for(tune_key(false, (size_t)H * W, n_views, maxcls));
    if (tc.edge_rows < 1) tc.edge_rows = tune_default.edge_rows;  // 0 (the fused form) is for batches
    FrameDesc f;
    describe_frame(&f, D, M, H, W, n_views, Ls, tc.edge_rows, th.thin);
    if (ws) {
        f.lists = ws->lists;
        f.counts = ws->counts;
        f.prefix = ws->prefix;
    } else {
        void *lists, *counts, *prefix;
        occl_status s = ensure("lists", list_entries(f, n_views) * sizeof(uint32_t), &lists);
        if (s != OCCL_OK) return s;
        s = ensure_zeroed("counts", kCountsBytes, &counts);
        if (s != OCCL_OK) return s;
        s = ensure("prefix", kPrefixInts * sizeof(int32_t), &prefix);
        if (s != OCCL_OK) return s;
        f.lists = (uint32_t*)lists;
        f.counts = (int32_t*)counts;
        f.prefix = (int32_t*)prefix;
    }
    hipEvent_t ev = ws ? nullptr : prof_begin(OCCL_STAGE_EDGES);
    hipError_t e = launch_edges(stream, f, n_views, vt, th.q_min);
    if (e != hipSuccess) return hip_fail(e, "edges");
    if (!ws) prof_end(OCCL_STAGE_EDGES, ev);
    if (!ws) ev = prof_begin(OCCL_STAGE_SCANLINES);
    // one scanline launch per register class present: K <= 2, then 4, 8, 16
    for (int ci = 0; ci < kNumClasses; ++ci) {
        if (f.cls_start[ci + 1] == f.cls_start[ci]) continue;
        e = launch_scanlines(stream, f, n_views, vt, th, ci, tc.scan_blocks_per_cu * n_cu);
        if (e != hipSuccess) return hip_fail(e, "scanlines");
    }
    if (ws) return OCCL_OK;
    prof_end(OCCL_STAGE_SCANLINES, ev);
    last_frame = f;
    last_views = n_views;
    last_vt = vt;
    last_th = th;
    last_scan_grid = tc.scan_blocks_per_cu * n_cu;
    return OCCL_OK;
}

extern "C" occl_status occl_time_scanlines(occl_ctx* ctx, int32_t reps, double* ms_per_pass) {
    if (!ctx || !ms_per_pass || reps < 1) return OCCL_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    const FrameDesc& f = ctx->last_frame;
    // the lists and prefix must still be the ones that call wrote
    auto li = ctx->bufs.find("lists");
    auto pr = ctx->bufs.find("prefix");
    if (ctx->last_views <= 0 || li == ctx->bufs.end() || pr == ctx->bufs.end() ||
        li->second.ptr != (void*)f.lists || pr->second.ptr != (void*)f.prefix)
        return ctx->fail(OCCL_ERR_STATE, "no exact-path frame to re-time");
    hipEvent_t a = ctx->take_event(), b = ctx->take_event();
    if (!a || !b) {
        if (a) ctx->ev_pool.push_back(a);
        if (b) ctx->ev_pool.push_back(b);
        return ctx->fail(OCCL_ERR_HIP, "hipEventCreate(time_scanlines)");
    }
    hipError_t e = hipEventRecord(a, ctx->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        for (int ci = 0; ci < kNumClasses && e == hipSuccess; ++ci) {
            if (f.cls_start[ci + 1] == f.cls_start[ci]) continue;
            e = launch_scanlines(ctx->stream, f, ctx->last_views, ctx->last_vt, ctx->last_th, ci,
                                 ctx->last_scan_grid);
        }
    if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    ctx->ev_pool.push_back(a);
    ctx->ev_pool.push_back(b);
    if (e != hipSuccess) return ctx->hip_fail(e, "time_scanlines");
    *ms_per_pass = (double)ms / reps;
    return OCCL_OK;
}

float occl::edge_q_min(float gamma) {
    if (gamma < 0.0f) return -INFINITY;
    // host sqrtf is the IEEE correctly rounded square root
    float q = gamma * gamma;
    while (q > 0.0f && std::sqrt(std::nextafter(q, 0.0f)) > gamma) q = std::nextafter(q, 0.0f);
    while (!(std::sqrt(q) > gamma)) q = std::nextafter(q, INFINITY);
    return q;
}

Thresholds occl::make_thresholds(const occl_params* p) {
    Thresholds th;
    th.gamma = p->edge_thr;
    th.q_min = edge_q_min(p->edge_thr);
    th.beta = p->disp_thr;
    th.zeta = p->dist_thr;
    int ns = (p->neighbours + 1) / 2;
    th.ns = ns < 1 ? 1 : ns;
    th.bilinear = (p->flags & OCCL_FLAG_BILINEAR) ? 1 : 0;
    th.thin = (p->flags & OCCL_FLAG_THIN) ? 1 : 0;
    return th;
}

namespace {
// occl_detect and occl_detect_routed: validation, view resolution, then the
// exact path, the exact path routed by the caller's logits, or (USE_CNN)
// the learned proposal followed by the routed exact path.
occl_status detect_impl(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                        const double* angles_deg, const float* ratios, const occl_params* params,
                        uint8_t* M, bool routed, const float* logits, uint8_t* tile_state) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    occl_status s = ctx->check_params(params, n_views, angles_deg, ratios);
    if (s != OCCL_OK) return s;
    if (routed && !(params->cnn_lo <= params->cnn_hi)) return ctx->fail(OCCL_ERR_INVALID_ARG, "cnn band");
    if (H < 0 || W < 0) return ctx->fail(OCCL_ERR_INVALID_ARG, "negative size");
    if ((size_t)H * (size_t)W > (size_t)1 << 31) return ctx->fail(OCCL_ERR_UNSUPPORTED, "frame too large");
    if ((size_t)H * W == 0 || n_views == 0) return OCCL_OK;
    if (!D || !M) return ctx->fail(OCCL_ERR_INVALID_ARG, "D or M is NULL");
    if (routed && !logits) return ctx->fail(OCCL_ERR_INVALID_ARG, "logits is NULL");
    if (H > 65535 || W > 65535) return ctx->fail(OCCL_ERR_UNSUPPORTED, "frame too large");
    const bool cnn = !routed && (params->flags & OCCL_FLAG_USE_CNN);
    if ((params->flags & OCCL_FLAG_THIN) && (routed || cnn))
        return ctx->fail(OCCL_ERR_UNSUPPORTED, "candidate thinning with routed tiles");
    if (cnn && !ctx->cnn_ready()) return ctx->fail(OCCL_ERR_NO_MODEL, "USE_CNN without loaded weights");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipSetDevice");
    ViewTable vt{};
    int Ls[OCCL_MAX_VIEWS];
    s = ctx->resolve_views(D, H, W, n_views, angles_deg, ratios, params, nullptr, &vt, Ls);
    if (s != OCCL_OK) return s;
    const Thresholds th = make_thresholds(params);
    if (routed)
        s = ctx->enqueue_routed(D, H, W, n_views, Ls, vt, th, params, logits, M, tile_state);
    else if (cnn)
        s = ctx->enqueue_frame_cnn(D, H, W, n_views, Ls, vt, th, params, M);
    else
        s = ctx->enqueue_frame(D, H, W, n_views, Ls, vt, th, M, nullptr);
    if (s != OCCL_OK) return s;
    if (params->flags & OCCL_FLAG_SYNC) {
        e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
    }
    return OCCL_OK;
}
}  // namespace

extern "C" occl_status occl_detect(occl_ctx* ctx, const float* D, int32_t H, int32_t W,
                                   int32_t n_views, const double* angles_deg, const float* ratios,
                                   const occl_params* params, uint8_t* M) {
    return detect_impl(ctx, D, H, W, n_views, angles_deg, ratios, params, M, false, nullptr, nullptr);
}

extern "C" occl_status occl_detect_routed(occl_ctx* ctx, const float* D, int32_t H, int32_t W,
                                          int32_t n_views, const double* angles_deg,
                                          const float* ratios, const occl_params* params,
                                          const float* logits, uint8_t* M, uint8_t* tile_state) {
    return detect_impl(ctx, D, H, W, n_views, angles_deg, ratios, params, M, true, logits, tile_state);
}

extern "C" occl_status occl_last_candidate_counts(occl_ctx* ctx, int64_t* out, int32_t n_views) {
    if (!ctx || !out) return OCCL_ERR_INVALID_ARG;
    if (ctx->last_views <= 0 || n_views != ctx->last_views)
        return ctx->fail(OCCL_ERR_STATE, "no matching previous occl_detect");
    (void)hipSetDevice(ctx->device);
    const FrameDesc& f = ctx->last_frame;
    const int C = f.ll.copies;
    std::vector<int32_t> h((size_t)n_views * C + 1);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpy(h.data(), f.prefix, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ctx->hip_fail(e, "prefix readback");
    for (int k = 0; k < n_views; ++k)  // prefix runs over views in vord order
        out[f.vord[k]] = (int64_t)h[(size_t)(k + 1) * C] - h[(size_t)k * C];
    return OCCL_OK;
}

extern "C" occl_status occl_edges(occl_ctx* ctx, const float* D, int32_t H, int32_t W, float* E,
                                  float* A) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (H < 0 || W < 0) return ctx->fail(OCCL_ERR_INVALID_ARG, "negative size");
    if ((size_t)H * W == 0 || (!E && !A)) return OCCL_OK;
    if (!D) return ctx->fail(OCCL_ERR_INVALID_ARG, "D is NULL");
    (void)hipSetDevice(ctx->device);
    hipError_t e = launch_edges_out(ctx->stream, D, H, W, E, A);
    if (e != hipSuccess) return ctx->hip_fail(e, "edges_out");
    return OCCL_OK;
}

extern "C" occl_status occl_zbuffer(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                                    const double* angles_deg, const float* ratios, float beta,
                                    uint8_t* M) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (H < 0 || W < 0 || n_views < 0 || n_views > OCCL_MAX_VIEWS || !std::isfinite(beta))
        return ctx->fail(OCCL_ERR_INVALID_ARG, "zbuffer arguments");
    if ((size_t)H * W == 0 || n_views == 0) return OCCL_OK;
    if (!D || !M || !angles_deg || !ratios) return ctx->fail(OCCL_ERR_INVALID_ARG, "NULL argument");
    if ((size_t)H * W > (size_t)1 << 31) return ctx->fail(OCCL_ERR_UNSUPPORTED, "frame too large");
    ViewTable vt{};
    for (int v = 0; v < n_views; ++v) {
        if (!std::isfinite(angles_deg[v]) || !std::isfinite(ratios[v]) || !(ratios[v] > 0.0f))
            return ctx->fail(OCCL_ERR_INVALID_ARG, "view");
        direction_of(angles_deg[v], &vt.c[v], &vt.s[v]);
        vt.r[v] = ratios[v];
    }
    (void)hipSetDevice(ctx->device);
    float mn, mx;
    uint32_t bad;
    occl_status s = ctx->d_stats(D, (size_t)H * W, &mn, &mx, &bad);
    if (s != OCCL_OK) return s;
    if (bad) return ctx->fail(OCCL_ERR_INVALID_ARG, "D holds non-finite values");
    const float amax = std::max(std::fabs(mn), std::fabs(mx));
    const long long cells = zbuffer_cells(H, W, n_views, ratios, amax);
    if (cells > (1ll << 32)) return ctx->fail(OCCL_ERR_UNSUPPORTED, "disparities too large for the target grid");
    void* best;
    s = ctx->ensure("zbuffer", (size_t)cells * sizeof(uint32_t), &best);
    if (s != OCCL_OK) return s;
    hipError_t e = launch_zbuffer(ctx->stream, D, H, W, n_views, vt, amax, beta, (uint32_t*)best, M);
    if (e != hipSuccess) return ctx->hip_fail(e, "zbuffer");
    return OCCL_OK;
}

extern "C" occl_status occl_median_fuse(occl_ctx* ctx, const float* maps, int32_t K, int32_t H,
                                        int32_t W, float* D) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    if (H < 0 || W < 0 || K < 1) return ctx->fail(OCCL_ERR_INVALID_ARG, "median arguments");
    if (K > 16) return ctx->fail(OCCL_ERR_UNSUPPORTED, "more than 16 maps");
    if ((size_t)H * W == 0) return OCCL_OK;
    if (!maps || !D) return ctx->fail(OCCL_ERR_INVALID_ARG, "NULL argument");
    (void)hipSetDevice(ctx->device);
    hipError_t e = launch_median_fuse(ctx->stream, maps, K, (long long)H * W, D);
    if (e != hipSuccess) return ctx->hip_fail(e, "median_fuse");
    return OCCL_OK;
}

extern "C" occl_status occl_confusion(occl_ctx* ctx, const uint8_t* pred, const uint8_t* ref,
                                      int64_t n, uint64_t* out) {
    if (!ctx || !out || n < 0) return OCCL_ERR_INVALID_ARG;
    if (n > 0 && (!pred || !ref)) return ctx->fail(OCCL_ERR_INVALID_ARG, "NULL mask");
    if (n == 0) {
        out[0] = out[1] = out[2] = out[3] = 0;
        return OCCL_OK;
    }
    (void)hipSetDevice(ctx->device);
    void* dev;
    occl_status s = ctx->ensure("confusion", (4 + 3 * (size_t)kConfusionBlocks) * sizeof(unsigned long long), &dev);
    if (s != OCCL_OK) return s;
    hipError_t e = launch_confusion(ctx->stream, pred, ref, (size_t)n, (unsigned long long*)dev);
    if (e != hipSuccess) return ctx->hip_fail(e, "confusion");
    e = hipMemcpyAsync(ctx->host_stats, dev, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                       ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return ctx->hip_fail(e, "confusion readback");
    std::memcpy(out, ctx->host_stats, 4 * sizeof(uint64_t));
    return OCCL_OK;
}

// Eq. (7): precision TP / (TP + FP), recall TP / (TP + FN), their harmonic
// mean F1 and IoU TP / (TP + FP + FN) of pred against ref, in double from
// the integer counts.  A ratio whose denominator is 0 has no errors to
// count and is 1 (F1 of P = R = 0 is 0).
extern "C" occl_status occl_quality(occl_ctx* ctx, const uint8_t* pred, const uint8_t* ref, int64_t n,
                                    double* out, uint64_t* counts) {
    if (!ctx || !out) return OCCL_ERR_INVALID_ARG;
    uint64_t c[4];
    occl_status s = occl_confusion(ctx, pred, ref, n, c);
    if (s != OCCL_OK) return s;
    const double tp = (double)c[0], fp = (double)c[1], fn = (double)c[2];
    const double P = (c[0] + c[1]) ? tp / (tp + fp) : 1.0;
    const double R = (c[0] + c[2]) ? tp / (tp + fn) : 1.0;
    out[0] = P;
    out[1] = R;
    out[2] = (P + R > 0.0) ? 2.0 * P * R / (P + R) : 0.0;
    out[3] = (c[0] + c[1] + c[2]) ? tp / (tp + fp + fn) : 1.0;
    if (counts) std::memcpy(counts, c, sizeof c);
    return OCCL_OK;
}
