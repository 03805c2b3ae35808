// occl_ctx.h -- the opaque context behind occl_ctx* (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "occl.h"
#include "occl_internal.h"

// Tuning bucket of a launch: batched or not, frame size class (log2 of the
// pixels), view count and the largest scan class.
inline uint64_t tune_key(bool batched, size_t pixels, int n_views, int max_class) {
    int lg = 0;
    while (lg < 62 && ((size_t)1 << (lg + 1)) <= pixels) ++lg;
    return (uint64_t)(batched ? 1 : 0) | ((uint64_t)lg << 1) | ((uint64_t)n_views << 8) |
           ((uint64_t)max_class << 16);
}

struct occl_ctx {
    struct Buf {
        void* ptr = nullptr;
        size_t bytes = 0;
    };

    int device = 0;
    int n_cu = 256;                      // compute units of the device
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::map<std::string, Buf> bufs;     // named device workspaces, grown on demand
    size_t workspace_cap = 0;            // 0 = unlimited
    void* scratch = nullptr;             // the device's static scratch array (occl_detect_noalloc),
                                         // its address resolved by occl_init
    uint32_t* host_stats = nullptr;      // pinned 64-byte staging area for read-backs
    std::string last_error;
    int last_views = 0;
    occl::FrameDesc last_frame{};        // layout of the most recent single-frame call
    occl::ViewTable last_vt{};           // its views, thresholds and scanline grid
    occl::Thresholds last_th{};
    int last_scan_grid = 0;

    // launch shapes: tuned per bucket (tune_key), default otherwise
    std::map<uint64_t, occl::TuneConfig> tuned;
    occl::TuneConfig tune_default{4, 8};
    occl::TuneConfig config_for(uint64_t key) const {
        auto it = tuned.find(key);
        return it == tuned.end() ? tune_default : it->second;
    }

    // batched path: frame table staging, graph cache, capture stream
    occl::FrameDesc* table_host = nullptr;  // pinned, kMaxBatch entries
    hipEvent_t table_event = nullptr;       // last upload from table_host
    std::vector<occl::FrameDesc> table_build;  // the table being built (zeroed entries)
    std::vector<uint8_t> table_cached;      // bytes of the last upload ...
    const void* table_cached_dev = nullptr; // ... and its device buffer (NULL: none known)
    // Uploads table_build[0 .. n) to dev on the stream unless the last upload
    // put the same bytes into the same buffer.
    occl_status upload_table(int n, void* dev);
    hipStream_t cap_stream = nullptr;       // graphs are captured here (never the null stream)
    hipStream_t cap_extra[occl::kMaxBatchBranches - 1] = {};  // further branches of a batch graph (capture only)
    hipEvent_t cap_fork = nullptr;                       // the batch graph's fork ...
    hipEvent_t cap_join[occl::kMaxBatchBranches - 1] = {};    // ... and joins
    struct GraphEntry {
        std::vector<uint8_t> sig;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;         // most recent first
    int64_t graph_builds = 0, graph_launches = 0;
    // the most recent batch's launch sequence (occl_time_batched re-runs it)
    struct LastBatch {
        bool valid = false;
        bool fused = false;                      // the batch took the fused pass
        const occl::FrameDesc* table = nullptr;  // device frame table
        unsigned* tickets = nullptr;             // the fused pass's tile tickets
        int n_branches = 0, n_views = 0, edge_rows = 0, edge_grid = 0, scan_grid = 0;
        int cut[occl::kMaxBatchBranches + 1] = {};
        int bstart[occl::kMaxBatchBranches + 1] = {};
        unsigned cls_mask[occl::kMaxBatchBranches] = {};
        occl::ViewTable vt{};
        occl::Thresholds th{};
    } last_batch;

    // learned tile proposal (k_cnn.hip); weights, Adam moments and
    // activations live in `bufs`
    bool cnn_loaded = false;
    int64_t cnn_step = 0;                // Adam steps taken
    const uint16_t* cnn_act[5] = {};     // outputs of layers 0..4 of the last forward pass
    int cnn_fwd_n = 0, cnn_fwd_h = 0, cnn_fwd_w = 0;  // its input shape (0: none yet)
    occl_status cnn_buffers(float** theta, uint16_t** wbf);
    occl_status cnn_layers(int first, const uint16_t* in, int N, int H, int W, float* Z);
    occl_status cnn_forward(const uint16_t* X, int N, int H, int W, float* Z);
    occl_status cnn_forward_frame(const float* D, int H, int W, int n_views, const occl::ViewTable& vt,
                                  const int* Ls, float* Z);
    occl_status cnn_backward(const uint16_t* X, int N, int H, int W, const float* T, double* loss);

    // stage profiling: event pairs per stage, resolved on occl_profile_read
    struct EvPair {
        int stage;
        hipEvent_t a, b;
    };
    bool profiling = false;
    std::vector<EvPair> ev_pairs;     // recorded, not yet resolved
    std::vector<hipEvent_t> ev_pool;  // free events
    double prof_ms[OCCL_N_STAGES] = {};
    int64_t prof_n[OCCL_N_STAGES] = {};
    hipEvent_t prof_begin(int stage);        // records and returns the start event (or null)
    void prof_end(int stage, hipEvent_t a);  // records the end event
    occl_status prof_resolve();
    hipEvent_t take_event();

    ~occl_ctx();
    void free_all();
    void drop_graphs();
    size_t total_bytes() const;
    occl_status ensure(const char* name, size_t bytes, void** out);
    occl_status ensure_zeroed(const char* name, size_t bytes, void** out);
    occl_status fail(occl_status s, const char* what);
    occl_status hip_fail(hipError_t e, const char* where);

    occl_status check_params(const occl_params* p, int n_views, const double* angles,
                             const float* ratios);
    // stats_ws: device workspace of (3 + 3 * kStatsBlocks) uint32 (NULL: the context's own)
    occl_status d_stats(const float* D, size_t n, float* mn, float* mx, uint32_t* bad,
                        void* stats_ws = nullptr);
    occl_status resolve_views(const float* D, int H, int W, int n_views, const double* angles,
                              const float* ratios, const occl_params* p, const int32_t* frame_L,
                              occl::ViewTable* vt, int* Ls, void* stats_ws = nullptr);
    // ws: the frame's workspace supplied by the caller (NULL: the context's
    // own buffers, grown on demand); a call with ws records no profiling
    // events and does not become the context's "most recent frame"
    occl_status enqueue_frame(const float* D, int H, int W, int n_views, const int* Ls,
                              const occl::ViewTable& vt, const occl::Thresholds& th, uint8_t* M,
                              const occl::TuneConfig* cfg, const occl::FrameWorkspace* ws = nullptr);
    occl_status enqueue_batch(int n_frames, const occl_frame* frames, int n_views, const int* Ls_all,
                              const occl::ViewTable& vt, const occl::Thresholds& th,
                              const occl::TuneConfig* cfg);
    // the fused pass takes batches whose views all have scanlines of at most
    // 128 samples, in the plain form (N = 1, nearest-pixel V)
    bool fusable(int n_views, int maxcls, const occl::Thresholds& th) const;
    occl_status enqueue_batch_fused(int n_frames, const occl_frame* frames, int n_views, const int* Ls_all,
                                    const occl::ViewTable& vt, const occl::Thresholds& th);

    bool cnn_ready() const { return cnn_loaded; }
    occl_status enqueue_frame_cnn(const float* D, int H, int W, int n_views, const int* Ls,
                                  const occl::ViewTable& vt, const occl::Thresholds& th,
                                  const occl_params* p, uint8_t* M);
    occl_status enqueue_routed(const float* D, int H, int W, int n_views, const int* Ls,
                               const occl::ViewTable& vt, const occl::Thresholds& th,
                               const occl_params* p, const float* logits, uint8_t* M,
                               uint8_t* tile_state);
};
