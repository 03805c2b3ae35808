// occl_internal.h -- declarations shared by the library's own HIP sources.
// Nothing here is part of the public ABI (include/occl.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "occl.h"

namespace occl {

// Edge pass block: 4 wavefronts, one 256-pixel row segment each (64 lanes x 4
// pixels), on 4 consecutive rows.
constexpr int kEdgeCols = 256;
constexpr int kEdgeRows = 4;
constexpr int kEdgeThreads = 256;

// Candidate lists.  The candidates of a view are split into `copies`
// segments by horizontal bands of edge-pass block rows; each segment has its
// own counter (on its own 128-byte line, so the appends of different bands
// never contend) and room for every pixel of its band (`cap`).  Entries are
// pixel indices y*W + x in no particular order: the mask is an OR of
// scanline hits, so the order never changes the result.
constexpr int kCounterPad = 32;    // int32 stride between counters (128 bytes)
constexpr int kMaxCopies = 64;
constexpr int kMaxSegments = 1024; // views x copies
// "counts" workspace: kMaxSegments padded counters, then the edge pass's
// completion counters (one top counter and kDoneGroups group counters); all
// are zero between frames.
constexpr int kDoneGroups = 32;
constexpr size_t kCountsBytes =
    ((size_t)kMaxSegments + 1 + kDoneGroups) * kCounterPad * sizeof(int32_t);

struct ListLayout {
    int copies;               // segments per view
    int block_rows_per_copy;  // edge-pass block rows feeding one segment
    size_t cap;               // entries per segment
};
ListLayout make_list_layout(int H, int W, int n_views);

// Per-view constants, passed by value as a kernel argument (copied at
// launch, so nothing on the host has to outlive the call).
struct ViewTable {
    float c[OCCL_MAX_VIEWS];   // cos(alpha), fp32 (octant-exact rule)
    float s[OCCL_MAX_VIEWS];   // sin(alpha)
    float r[OCCL_MAX_VIEWS];   // baseline ratio
    int h[OCCL_MAX_VIEWS];     // half scan length floor(L/2)
};

struct Thresholds {
    float gamma;   // edge threshold (Eq. 2)
    float q_min;   // smallest fp32 q with sqrt_rn(q) > gamma (edge_q_min)
    float beta;    // disparity threshold (Eq. 5)
    float zeta;    // distance threshold (Eq. 5)
    int ns;        // neighbours per side, max(1, ceil(N/2))
};

// Smallest K (power of two, 1..16) with 64*K >= n samples.
__host__ __device__ inline int lanes_per_scanline_k(int n) {
    int k = 1;
    while (64 * k < n) k <<= 1;
    return k;
}

// ---- launchers (k_exact.hip) ------------------------------------------------
hipError_t launch_edges_candidates(hipStream_t st, const float* D, int H, int W, uint8_t* M,
                                   int n_views, const ViewTable& vt, float q_min,
                                   const ListLayout& ll, uint32_t* lists, int32_t* counts,
                                   int32_t* prefix);

// Smallest fp32 q >= 0 whose correctly rounded square root exceeds gamma
// (-inf when gamma < 0: every magnitude passes).  Host only.
float edge_q_min(float gamma);

// Thresholds of a validated occl_params (host only).
Thresholds make_thresholds(const occl_params* p);

// Processes the scanlines of every candidate of the views listed in `views`.
// kclass 2 serves the views whose scanlines fit K = 1 or 2 samples per lane;
// kclass 4, 8, 16 serve exactly that K.
hipError_t launch_scanlines(hipStream_t st, const float* D, int H, int W, uint8_t* M,
                            const ViewTable& vt, const Thresholds& th, const int* views,
                            int n_list, int kclass, const ListLayout& ll, const uint32_t* lists,
                            const int32_t* prefix, int n_blocks);

// min / max / non-finite count of D into dev[0..2] (orderable uint32 / count).
hipError_t launch_scan_stats(hipStream_t st, const float* D, size_t n, uint32_t* dev);

hipError_t launch_edges_out(hipStream_t st, const float* D, int H, int W, float* E, float* A);

hipError_t launch_confusion(hipStream_t st, const uint8_t* pred, const uint8_t* ref, size_t n,
                            unsigned long long* dev4);

}  // namespace occl
