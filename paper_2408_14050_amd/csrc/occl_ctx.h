// occl_ctx.h -- the opaque context behind occl_ctx* (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "occl.h"
#include "occl_internal.h"

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
    uint32_t* host_stats = nullptr;      // pinned 64-byte staging area for read-backs
    std::string last_error;
    int last_H = 0, last_W = 0, last_views = 0;

    // learned tile proposal (k_cnn.hip); weights live in `bufs`
    bool cnn_loaded = false;

    // stage profiling: event pairs per stage, resolved on occl_profile_read
    struct EvPair {
        int stage;
        hipEvent_t a, b;
    };
    bool profiling = false;
    std::vector<EvPair> ev_pairs;     // recorded, not yet resolved
    std::vector<hipEvent_t> ev_pool;  // free events
    double prof_ms[OCCL_N_STAGES] = {0, 0, 0, 0};
    int64_t prof_n[OCCL_N_STAGES] = {0, 0, 0, 0};
    hipEvent_t prof_begin(int stage);        // records and returns the start event (or null)
    void prof_end(int stage, hipEvent_t a);  // records the end event
    occl_status prof_resolve();
    hipEvent_t take_event();

    ~occl_ctx();
    void free_all();
    size_t total_bytes() const;
    occl_status ensure(const char* name, size_t bytes, void** out);
    occl_status ensure_zeroed(const char* name, size_t bytes, void** out);
    occl_status fail(occl_status s, const char* what);
    occl_status hip_fail(hipError_t e, const char* where);

    occl_status check_params(const occl_params* p, int n_views, const double* angles,
                             const float* ratios);
    occl_status d_stats(const float* D, size_t n, float* mn, float* mx, uint32_t* bad);
    occl_status resolve_views(const float* D, int H, int W, int n_views, const double* angles,
                              const float* ratios, const occl_params* p, const int32_t* frame_L,
                              occl::ViewTable* vt, int* Ls);
    occl_status enqueue_frame(const float* D, int H, int W, int n_views, const occl::ViewTable& vt,
                              const occl::Thresholds& th, uint8_t* M);

    bool cnn_ready() const { return cnn_loaded; }
    occl_status enqueue_frame_cnn(const float* D, int H, int W, int n_views,
                                  const occl::ViewTable& vt, const occl::Thresholds& th,
                                  const occl_params* p, uint8_t* M);
};
