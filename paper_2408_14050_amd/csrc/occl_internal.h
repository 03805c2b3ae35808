// occl_internal.h -- declarations shared by the library's own HIP sources.
// Nothing here is part of the public ABI (include/occl.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "occl.h"

namespace occl {

// Edge pass: one wavefront per 256-pixel row segment (64 lanes x 4 pixels);
// a block stacks `edge_rows` (1..kMaxEdgeRows, tuned) wavefronts on
// consecutive rows.
constexpr int kEdgeCols = 256;
constexpr int kMaxEdgeRows = 16;

// Candidate lists.  The candidates of a view are split into `copies`
// segments by horizontal bands of edge-pass block rows; each segment has its
// own counter (on its own 128-byte line, so the appends of different bands
// never contend) and room for every pixel of its band (`cap`).  Entries are
// packed pixel coordinates (y << 16) | x in no particular order: the mask is
// an OR of scanline hits, so the order never changes the result.
constexpr int kCounterPad = 32;    // int32 stride between counters (128 bytes)
constexpr int kMaxCopies = 64;
#ifndef OCCL_WAVES_PER_BAND
#define OCCL_WAVES_PER_BAND 200
#endif
constexpr int kWavesPerBand = OCCL_WAVES_PER_BAND;  // edge-pass wavefronts per list segment (target)
constexpr int kMaxSegments = 1024; // views x copies
// Per-frame "counts" workspace: kMaxSegments padded counters, then the edge
// pass's completion counters (one top counter and kDoneGroups group
// counters); all are zero between frames.
constexpr int kDoneGroups = 32;
constexpr size_t kCountsInts = ((size_t)kMaxSegments + 1 + kDoneGroups) * kCounterPad;
constexpr size_t kCountsBytes = kCountsInts * sizeof(int32_t);
constexpr size_t kPrefixInts = kMaxSegments + 1;

// Scanline register classes: a scanline of n samples keeps K = 1, 2, 4, 8 or
// 16 samples per lane; class 0 serves K = 1 and 2, classes 1..3 serve 4, 8, 16.
constexpr int kNumClasses = 4;
constexpr int kMaxBatch = 1024;
// Graph branches of a batched launch (frames split by pixel count).
#ifndef OCCL_BATCH_BRANCHES
#define OCCL_BATCH_BRANCHES 2
#endif
constexpr int kMaxBatchBranches = 4;
constexpr int kBatchBranches = OCCL_BATCH_BRANCHES;
static_assert(kBatchBranches >= 1 && kBatchBranches <= kMaxBatchBranches, "batch branches");

// Smallest K (power of two, 1..16) with 64*K >= n samples.
__host__ __device__ inline int lanes_per_scanline_k(int n) {
    int k = 1;
    while (64 * k < n) k <<= 1;
    return k;
}
// Class of a scanline of at most n samples.
__host__ __device__ inline int scan_class_n(int n) {
    const int K = lanes_per_scanline_k(n);
    return K <= 2 ? 0 : (K == 4 ? 1 : (K == 8 ? 2 : 3));
}
// Longest scanline of a view with half length h: 2h + 1 samples, 3h + 1
// with candidate thinning (a merged window reaches h further).
__host__ __device__ inline int view_samples(int h, int thin) { return thin ? 3 * h + 1 : 2 * h + 1; }
__host__ __device__ inline int scan_class(int h, int thin = 0) { return scan_class_n(view_samples(h, thin)); }

// Per-view constants shared by every frame of a call, passed by value as a
// kernel argument (copied at launch, so nothing on the host has to outlive
// the call).
struct ViewTable {
    float c[OCCL_MAX_VIEWS];   // cos(alpha), fp32 (octant-exact rule)
    float s[OCCL_MAX_VIEWS];   // sin(alpha)
    float r[OCCL_MAX_VIEWS];   // baseline ratio
};

struct Thresholds {
    float gamma;   // edge threshold (Eq. 2)
    float q_min;   // smallest fp32 q with sqrt_rn(q) > gamma (edge_q_min)
    float beta;    // disparity threshold (Eq. 5)
    float zeta;    // distance threshold (Eq. 5)
    int ns;        // neighbours per side, max(1, ceil(N/2))
    int bilinear;  // 1: V by bilinear interpolation at the real sample position (variant)
    int thin;      // 1: candidate thinning (variant; single frames, not routed)
};

struct ListLayout {
    int copies;               // segments per view
    int block_rows_per_copy;  // edge-pass block rows feeding one segment
    int edge_rows;            // rows (wavefronts) per edge-pass block
    size_t cap;               // entries per segment
};
ListLayout make_list_layout(int H, int W, int n_views, int edge_rows);

// One frame as the kernels see it.  The prefix array holds the exclusive
// prefix of the segment sizes in class-major order: the views of class 0 in
// `vord` order, then class 1, ...; bands inner.
struct FrameDesc {
    const float* D;
    uint8_t* M;
    int H, W;
    ListLayout ll;
    uint32_t* lists;
    int32_t* counts;
    int32_t* prefix;
    uint32_t copies_magic;            // ceil(2^32 / ll.copies) for copies > 1: umulhi(j, magic) = j / copies
                                      // for j < 2^16
    int gx, gy;                       // edge-pass blocks along x / y
    int block_begin;                  // first flat edge-pass block (batched launch)
    int h[OCCL_MAX_VIEWS];            // half scan length floor(L/2) per view
    int vord[OCCL_MAX_VIEWS];         // views ordered by scan class (stable)
    int cls_start[kNumClasses + 1];   // number of views of class < ci in vord
};

constexpr int kTile = 16;

// Launch shape chosen by the autotuner.
struct TuneConfig {
    int edge_rows;           // 1..16
    int scan_blocks_per_cu;  // persistent scanline blocks per compute unit
};

// Workspace of one frame's exact path: candidate lists (list_entries(f)
// uint32), the segment and completion counters (kCountsInts int32, all zero
// between frames) and the class-major prefix (kPrefixInts int32).
struct FrameWorkspace {
    uint32_t* lists;
    int32_t* counts;
    int32_t* prefix;
};
inline size_t list_entries(const FrameDesc& f, int n_views) {
    return f.ll.cap * (size_t)f.ll.copies * (size_t)n_views;
}

// Address of this device's static scratch array (occl_noalloc.hip); called
// by occl_init with `device` current, once per device.
occl_status scratch_resolve(int device, void** out);

// Fills the fields of a FrameDesc that depend only on sizes and scan lengths
// (layout, grid, class order); the workspace pointers are set by the caller.
void describe_frame(FrameDesc* f, const float* D, uint8_t* M, int H, int W, int n_views,
                    const int* Ls, int edge_rows, int thin = 0);

// ---- launchers (k_exact.hip) ------------------------------------------------
hipError_t launch_edges(hipStream_t st, const FrameDesc& f, int n_views, const ViewTable& vt,
                        float q_min);
hipError_t launch_scanlines(hipStream_t st, const FrameDesc& f, int n_views, const ViewTable& vt,
                            const Thresholds& th, int cls, int n_blocks);
// Resident blocks per CU of the batched edge pass at this block height (its
// persistent grid must not exceed what fits at once).
int edges_batched_blocks_per_cu(int edge_rows);
hipError_t launch_edges_batched(hipStream_t st, const FrameDesc* table, int n_frames,
                                int total_blocks, int n_views, const ViewTable& vt, float q_min,
                                int edge_rows, int n_blocks);
hipError_t launch_scanlines_batched(hipStream_t st, const FrameDesc* table, int n_frames,
                                    int n_views, const ViewTable& vt, const Thresholds& th,
                                    int cls, int n_blocks);

// Fused pass (k_fused, after k_clear_masks): every view of every frame in
// one persistent launch, for frames whose views all have scanlines of at
// most 128 samples, the plain form (N = 1, nearest-pixel V, no routed tiles,
// no thinning) and at most kFusedMaxViews views.  Frames are described with
// tiles of kFusedTileRows rows x kEdgeCols columns (describe_frame with
// edge_rows = kFusedTileRows; block_begin = first flat tile).  tickets:
// kFusedParts counters 128 bytes apart (cleared by the launch itself).
#ifndef OCCL_FUSED_ROWS
#define OCCL_FUSED_ROWS 16
#endif
constexpr int kFusedTileRows = OCCL_FUSED_ROWS;  // rows (wavefronts) per tile, at most 16
static_assert(kFusedTileRows >= 1 && kFusedTileRows <= 16, "fused tile rows");
constexpr int kClearChunkBytes = 65536;  // bytes of mask per block of the mask fill
constexpr int kFusedTickets = 8 * 32;  // uint32 of the tickets buffer
constexpr int kFusedMaxViews = 64;
int fused_blocks_per_cu();
// one kernel of the fused form: stage 0 the mask fill, stage 1 the fused pass
hipError_t launch_fused_stage(hipStream_t st, const FrameDesc* table, int n_frames, int total_tiles, int n_views,
                              const ViewTable& vt, const Thresholds& th, unsigned* tickets, int n_blocks,
                              int clear_blocks, int stage);
hipError_t launch_fused(hipStream_t st, const FrameDesc* table, int n_frames, int total_tiles, int n_views,
                        const ViewTable& vt, const Thresholds& th, unsigned* tickets, int n_blocks,
                        int clear_blocks);

// Smallest fp32 q >= 0 whose correctly rounded square root exceeds gamma
// (-inf when gamma < 0: every magnitude passes).  Host only.
float edge_q_min(float gamma);

// Thresholds of a validated occl_params (host only).
Thresholds make_thresholds(const occl_params* p);

// ---- helpers (k_util.hip) ---------------------------------------------------
// min / max / non-finite count of D into dev[0..2] (orderable uint32 / count).
// min / max (orderable uints) and non-finite count of D into dev[0..2]; dev
// holds 3 + 3 * kStatsBlocks uint32
constexpr int kStatsBlocks = 1024;
hipError_t launch_scan_stats(hipStream_t st, const float* D, size_t n, uint32_t* dev);

// p[0 .. n) = 0 (a fill kernel: no memset node ever enters a captured graph)
hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, long long n);

hipError_t launch_edges_out(hipStream_t st, const float* D, int H, int W, float* E, float* A);

// Tile states from logits z (n entries): 0 if z < z_lo, 1 if z > z_hi, else
// 2 (NaN included).
hipError_t launch_route_state(hipStream_t st, const float* logits, size_t n, float z_lo, float z_hi,
                              uint8_t* tstate);
// M[v][y][x] = state of its tile wherever that state is 0 or 1.
hipError_t launch_route_apply(hipStream_t st, const uint8_t* tstate, int n_views, int H, int W, int tiles_y,
                              int tiles_x, uint8_t* M);


// Forward-warping ground truth: M[v][y][x] = 1 iff some pixel lands on the
// same nearest target pixel of view v with a disparity larger by more than
// beta.  best: workspace of zbuffer_cells(...) uint32; max_abs_d >= max |D|.
long long zbuffer_cells(int H, int W, int n_views, const float* ratios, float max_abs_d);
hipError_t launch_zbuffer(hipStream_t st, const float* D, int H, int W, int n_views, const ViewTable& vt,
                          float max_abs_d, float beta, uint32_t* best, uint8_t* M);

// D[i] = NaN-ignoring median of maps[k][i], k < K (1..16).
hipError_t launch_median_fuse(hipStream_t st, const float* maps, int K, long long n, float* D);

// TP, FP, FN, TN of two masks into dev[0..3]; dev holds 4 + 3 * kConfusionBlocks
// entries (the rest is scratch for per-block partials).
constexpr int kConfusionBlocks = 1024;
hipError_t launch_confusion(hipStream_t st, const uint8_t* pred, const uint8_t* ref, size_t n,
                            unsigned long long* dev4);

}  // namespace occl
