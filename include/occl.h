/*
 * occl.h -- C ABI of the MI355X (gfx950) fast edge-aware occlusion detector.
 *
 * Method: Sippel, Seiler, Kaup, "Fast Edge-Aware Occlusion Detection in the
 * Context of Multispectral Camera Arrays", ICIP 2024, Sec. 3, Eqs. (1)-(6).
 * From the fused centre-view disparity map D the library computes the edge
 * maps (Eq. 1), keeps the edge candidates that face each peripheral camera
 * (Eq. 2), samples a scanline of 2*floor(L/2)+1 pixels along the camera's
 * baseline through every candidate (Eq. 4), warps the samples into the
 * peripheral view (W = g - r*V), sorts them, compares each sorted sample
 * with its sorted neighbours (Eq. 5) and sets the occluded pixels of the
 * per-view mask M (Eq. 6).
 *
 * Conventions (the readings of the paper the library implements):
 *  - D is fp32, row-major [H][W], x to the right, y down.
 *  - A view is given by the angle (degrees, double) of the baseline from the
 *    centre camera to the peripheral camera, measured from +x towards +y,
 *    and the baseline ratio r > 0 (disparity in that view = r * D).
 *  - The direction vector (cos, sin) of an angle is computed on the host in
 *    double for the octant reference angle in (0, 45] degrees and rounded to
 *    fp32; multiples of 90 degrees are exact.
 *  - E_x, E_y are forward differences, zero on the last column / row;
 *    a pixel is a candidate iff sqrt(E_x^2 + E_y^2) > gamma and
 *    E_x*cos + E_y*sin > 0 (fp32, no fused multiply-add).
 *  - Scanline coordinates: fp32 multiply then add, round half to even;
 *    samples outside the frame are dropped.
 *  - Sort ascending by W, ties by ascending offset g; a sorted sample k is
 *    occluded iff for some d in +-1..+-max(1, ceil(N/2)):
 *    |W_k - W_{k+d}| < zeta and V_{k+d} - V_k > beta.
 *  - M[v][y][x] in {0, 1}, view-major, 1 = occluded in view v.
 *
 * Memory: D and M are device pointers owned by the caller; the library
 * never allocates or frees them and only reads D / writes M on the
 * context's stream.  They must stay valid until that stream's work is done.
 * Every call is asynchronous on the context's stream unless stated.
 *
 * Errors: every function returns an occl_status.  Argument validation runs
 * before anything is enqueued; a rejected call has no side effects.
 * Asynchronous device faults surface at the next call or at occl_sync.  A
 * context is not thread-safe: use one context per stream.
 */
#ifndef OCCL_H
#define OCCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct occl_ctx occl_ctx;

typedef enum {
    OCCL_OK = 0,
    OCCL_ERR_INVALID_ARG = -1,   /* bad pointer, size, angle, ratio, threshold ... */
    OCCL_ERR_OUT_OF_MEMORY = -2, /* workspace allocation failed or exceeds the cap */
    OCCL_ERR_HIP = -3,           /* a HIP runtime call failed (message: occl_last_error) */
    OCCL_ERR_UNSUPPORTED = -4,   /* e.g. resolved scan length L > OCCL_MAX_SCAN_LEN */
    OCCL_ERR_NO_MODEL = -5,      /* the learned tile proposal was requested without weights */
    OCCL_ERR_STATE = -6          /* call not valid in the context's current state */
} occl_status;

#define OCCL_MAX_VIEWS 64
#define OCCL_MAX_SCAN_LEN 1023
#define OCCL_MAX_NEIGHBOURS 64

/* flags of occl_params */
#define OCCL_FLAG_SYNC 1u            /* synchronise the stream before returning */
#define OCCL_FLAG_VALIDATE_INPUT 2u  /* check D for non-finite values first (synchronises) */
#define OCCL_FLAG_USE_CNN 4u         /* learned tile proposal + exact fallback (needs weights) */
#define OCCL_FLAG_BILINEAR 8u        /* variant: V read by bilinear interpolation of D at the real
                                        scanline position (taps clamped into the frame; top row,
                                        bottom row, then vertical blend, fp32 without FMA); kept
                                        samples and marked pixels stay the nearest pixels */
#define OCCL_FLAG_THIN 16u           /* variant, an approximation of the method (the thinner
                                        candidate list the paper's summary, Sec. 6, leaves for
                                        future work): a candidate whose scanline pixel at g = -1 is
                                        a candidate of the same view (Eq. 2) is not scanned; every
                                        other candidate scans g = -h .. h + m, m = the number of
                                        consecutive candidates at g = 1, 2, ... (at most h; a pixel
                                        outside the frame ends the run).  occl_detect only, without
                                        OCCL_FLAG_USE_CNN (else OCCL_ERR_UNSUPPORTED); L at most
                                        OCCL_THIN_MAX_SCAN_LEN.  Composes with N and bilinear V. */
#define OCCL_THIN_MAX_SCAN_LEN 683   /* 3 * floor(L / 2) + 1 <= 1024 samples per scanline */

/* Detector parameters (Sec. 3: gamma of Eq. 2, zeta and beta of Eq. 5,
 * N of Eq. 5, L of Eqs. 3-4). */
typedef struct {
    uint32_t struct_size;        /* must be sizeof(occl_params) */
    float edge_thr;              /* gamma, px (> 0 is usual; any finite value accepted) */
    float disp_thr;              /* beta, px, finite */
    float dist_thr;              /* zeta, px, finite */
    int32_t neighbours;          /* N, 1..OCCL_MAX_NEIGHBOURS */
    int32_t scan_len;            /* L > 0: the same L for every view;
                                    0: per view L = ceil(max(D) * r) + 2 (fp32 product);
                                   -1: per view L = ceil(2 * r * (max(D) - min(D))) (Eq. 3
                                       with the ratio).  0 and -1 read max/min of D back
                                       to the host, so the call synchronises. */
    const int32_t* scan_len_per_view; /* optional host array [n_views]; overrides scan_len */
    uint32_t flags;              /* OCCL_FLAG_* */
    float cnn_lo, cnn_hi;        /* tile-probability band that falls back to the exact path */
} occl_params;

/* Fills *p with the defaults gamma = 1, beta = 0.5, zeta = 1, N = 1, L = 0,
 * no flags, band [0.05, 0.95]. */
void occl_params_default(occl_params* p);

/* Creates a context on HIP device `device`.  `hip_stream` is the hipStream_t
 * every call of this context is enqueued on; NULL: the context creates a
 * stream of its own (default priority, ordered with the device's null
 * stream like any blocking stream) and destroys it in occl_release.  All work
 * is enqueued on that stream; the library's other streams serve only to
 * capture the batched launch's graph.  The hints size the initial workspace
 * (0: grow on first use).  The context owns its workspaces, tuned launch
 * shapes, graphs and network state; it also resolves the address of the
 * device's static scratch array used by occl_detect_noalloc. */
occl_status occl_init(occl_ctx** out, int device, void* hip_stream, size_t max_pixels_hint,
                      int32_t max_views_hint);

/* Upper bound on the device memory the context's workspaces may hold in total
 * (bytes; 0 = unlimited, the default).  A call whose workspace would grow
 * beyond it returns OCCL_ERR_OUT_OF_MEMORY before anything is enqueued; what
 * is already allocated stays.  occl_workspace_bytes reports the current
 * total. */
occl_status occl_set_workspace_cap(occl_ctx* ctx, size_t bytes);
occl_status occl_workspace_bytes(const occl_ctx* ctx, size_t* bytes);

/* One frame, n_views views.
 *   D          device fp32 [H][W], row-major contiguous (16-byte alignment and W % 4 == 0
 *              select the vectorised path; anything else is still correct)
 *   H, W       0..65535 (larger: OCCL_ERR_UNSUPPORTED); H*W == 0 or n_views == 0 is a valid
 *              empty call (nothing enqueued)
 *   n_views    0..OCCL_MAX_VIEWS
 *   angles_deg host double [n_views], finite
 *   ratios     host float [n_views], finite and > 0
 *   params     host occl_params
 *   M          device uint8 [n_views][H][W]; every byte is written with 0 or 1 */
occl_status occl_detect(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                        const double* angles_deg, const float* ratios, const occl_params* params,
                        uint8_t* M);

/* ---- the exact path without device allocation ----------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * occl_detect_noalloc writes exactly the masks occl_detect writes (the same
 * kernels and launch shape) but takes the frame's workspace (candidate
 * lists, counters, prefix, statistics partials) from a static device array
 * of OCCL_NOALLOC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends; its address is resolved by occl_init.
 * The call itself allocates nothing: no hipMalloc, hipFree or allocating
 * library routine.
 * Limits: the candidate lists need about 4 * n_views * H * W bytes (plus
 * 160 KiB of counters): a 1280 x 960 frame with 8 views fits; a frame that
 * does not fit returns OCCL_ERR_UNSUPPORTED (occl_last_error gives both
 * sizes) with nothing enqueued, except that a scan_len of 0 or -1 first
 * reads D's statistics (through the array) and synchronises, as occl_detect
 * does.  OCCL_FLAG_USE_CNN returns OCCL_ERR_UNSUPPORTED.
 * Sharing: every call on one device uses that device's one array and leaves
 * its contents there; the counters that must start at zero are cleared at
 * the start of each call.  Calls that overlap on one device (several
 * streams or contexts) race: the caller serialises them.
 * The arguments are those of occl_detect. */
#define OCCL_NOALLOC_SCRATCH_BYTES (64ull * 1024ull * 1024ull)
occl_status occl_detect_noalloc(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                                const double* angles_deg, const float* ratios,
                                const occl_params* params, uint8_t* M);

/* A frame of a batch: its own size, mask and optionally its own scan lengths
 * (host array [n_views]; NULL: params->scan_len / scan_len_per_view). */
typedef struct {
    const float* D;
    int32_t H, W;
    uint8_t* M;
    const int32_t* scan_len_per_view;
} occl_frame;

/* Many frames of uneven size with the same views, in one graph launch on
 * the context's stream.  The launch shape is taken from the autotuner
 * cache.  Per-frame semantics are exactly those of occl_detect. */
occl_status occl_detect_batched(occl_ctx* ctx, int32_t n_frames, const occl_frame* frames,
                                int32_t n_views, const double* angles_deg, const float* ratios,
                                const occl_params* params);

/* Launch shape of the exact path: edge-pass rows (wavefronts) per block and
 * persistent scanline blocks per compute unit. */
typedef struct {
    int32_t edge_rows;           /* 1, 2, 4, 8 or 16 */
    int32_t scan_blocks_per_cu;  /* 1..64 */
    float ms;                    /* measured time per call of the chosen shape (autotune output) */
} occl_tune;

/* Autotuner: times the candidate launch shapes on this frame (each trial
 * computes the full masks into M, so M ends with the correct result) and
 * records the fastest for frames of the same size class (log2 of H*W), view
 * count and scan class; later calls in that bucket use it.  `reps` timed
 * calls per shape (<= 0: 10).  `out` (optional) receives the choice.
 * Synchronises the stream. */
occl_status occl_autotune(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                          const double* angles_deg, const float* ratios, const occl_params* params,
                          uint8_t* M, int32_t reps, occl_tune* out);

/* The same for a batch (1..1024 non-empty frames); the bucket is the batch's
 * total pixel count, view count and scan class. */
occl_status occl_autotune_batched(occl_ctx* ctx, int32_t n_frames, const occl_frame* frames,
                                  int32_t n_views, const double* angles_deg, const float* ratios,
                                  const occl_params* params, int32_t reps, occl_tune* out);

/* Writes / reads the tuned launch shapes as text ("bucket edge_rows
 * scan_blocks_per_cu" per line).  Loading validates every line and merges
 * the entries into the context; a malformed file changes nothing. */
occl_status occl_tune_save(const occl_ctx* ctx, const char* path);
occl_status occl_tune_load(occl_ctx* ctx, const char* path);

/* Candidates per view of the most recent occl_detect (host int64 [n_views]);
 * synchronises the stream. */
occl_status occl_last_candidate_counts(occl_ctx* ctx, int64_t* out, int32_t n_views);

/* Edge magnitude E and angle A = atan2(E_y, E_x) of Eq. (1) (device fp32 [H][W] each;
 * either may be NULL). */
occl_status occl_edges(occl_ctx* ctx, const float* D, int32_t H, int32_t W, float* E, float* A);

/* Confusion counts of two masks (Eq. 7 inputs): pred, ref device uint8 [n];
 * out host uint64[4] = {TP, FP, FN, TN}; synchronises the stream. */
occl_status occl_confusion(occl_ctx* ctx, const uint8_t* pred, const uint8_t* ref, int64_t n,
                           uint64_t* out);

/* Quality of pred against ref by Eq. (7): out host double[4] = {precision
 * TP/(TP+FP), recall TP/(TP+FN), F1 = 2PR/(P+R), IoU TP/(TP+FP+FN)} from the
 * counts of occl_confusion (a ratio with a zero denominator is 1; F1 with
 * P = R = 0 is 0); counts (host uint64[4], may be NULL) receives {TP, FP, FN,
 * TN}.  Synchronises the stream. */
occl_status occl_quality(occl_ctx* ctx, const uint8_t* pred, const uint8_t* ref, int64_t n,
                         double* out, uint64_t* counts);

/* ---- learned tile proposal + exact fallback -------------------------------
 * Not part of the paper: a small network proposes, per 16 x 16 pixel tile
 * and view, the probability that the tile holds occluded pixels (the tile's
 * occluded fraction of the exact mask of Sec. 3 is its training target).
 * Confident tiles are filled, the rest keep the mask of the exact path of
 * Sec. 3 (run over the frame: confident tiles hold no candidates in
 * practice, so restricting it saves nothing).  Network: six 3x3 convolutions 8->32 (stride 2),
 * 32->32 (2), 32->32 (2), 32->32 (2), 32->32 (1), 32->1 (1), ReLU after all
 * but the last; bf16 weights and activations, fp32 accumulation and logits.
 * Parameters are one flat fp32 vector, layer by layer, each layer's weights
 * [Cout][3][3][Cin] then its biases [Cout]. */

/* Number of parameters of the network (39617). */
size_t occl_cnn_num_params(void);

/* Random initial weights (He-uniform from `seed`, zero biases), zero Adam
 * state, step 0. */
occl_status occl_cnn_init(occl_ctx* ctx, uint64_t seed);

/* Model state for checkpoint / resume: parameters, Adam moments m and v
 * (host fp32 [n] each; m, v may be NULL on set = zero, on get = skipped) and
 * the Adam step count.  n must equal occl_cnn_num_params(); set rejects
 * non-finite values with OCCL_ERR_INVALID_ARG and leaves the state as it was. */
occl_status occl_cnn_set_state(occl_ctx* ctx, const float* theta, const float* m, const float* v,
                               int64_t step, size_t n);
occl_status occl_cnn_get_state(occl_ctx* ctx, float* theta, float* m, float* v, int64_t* step,
                               size_t n);

/* Network input of every view: device bf16 X [n_views][H][W][8] with the
 * channels D * r / L, E / 8, cos A, sin A, cos alpha, sin alpha, r / 2, 0
 * (E and A = atan2(E_y, E_x) of Eq. (1); (cos alpha, sin alpha) the view's
 * direction; scan_len host int32 [n_views] >= 1). */
occl_status occl_cnn_pack(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                          const double* angles_deg, const float* ratios, const int32_t* scan_len,
                          uint16_t* X);

/* Logits of N inputs X (device bf16 [N][H][W][8]) into device fp32
 * logits [N][ceil(H/16)][ceil(W/16)].  Needs weights (OCCL_ERR_NO_MODEL). */
occl_status occl_cnn_forward(occl_ctx* ctx, const uint16_t* X, int32_t N, int32_t H, int32_t W,
                             float* logits);

/* The proposal of one frame: logits of every view straight from D (device
 * fp32 [H][W]) into device fp32 logits [n_views][ceil(H/16)][ceil(W/16)].
 * The input packing is fused into the first layer; the logits are
 * bit-identical to occl_cnn_pack followed by occl_cnn_forward with the same
 * views and scan lengths (host int32 [n_views] >= 1).  Needs weights. */
occl_status occl_cnn_propose(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                             const double* angles_deg, const float* ratios, const int32_t* scan_len,
                             float* logits);

/* Copies the output of hidden layer `layer` (0..4) of the most recent
 * forward pass (occl_cnn_forward, _backward, _train_step, _propose or a
 * USE_CNN detection; the last two keep no layer-0 output: OCCL_ERR_STATE)
 * into dst: device bf16 [N][H_l][W_l][32] with n =
 * N * H_l * W_l * 32 elements (H_l = H halved, rounding up, once per
 * stride-2 layer up to `layer`).  For inspection and tests. */
occl_status occl_cnn_activation(occl_ctx* ctx, int32_t layer, uint16_t* dst, size_t n);

/* Mean soft binary cross-entropy of the logits against targets T (device fp32,
 * same shape as the logits, values in [0, 1]) and its gradient.  `loss`
 * (host, may be NULL) receives the loss; `grad` (host fp32
 * [occl_cnn_num_params()], may be NULL) the gradient.  Synchronises when
 * either is requested. */
occl_status occl_cnn_backward(occl_ctx* ctx, const uint16_t* X, int32_t N, int32_t H, int32_t W,
                              const float* T, double* loss, float* grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * learning rate lr > 0 on the gradient of occl_cnn_backward's loss. */
occl_status occl_cnn_train_step(occl_ctx* ctx, const uint16_t* X, int32_t N, int32_t H, int32_t W,
                                const float* T, float lr, double* loss);

/* Training targets: the occluded fraction of every 16 x 16 tile (tiles
 * aligned to (0, 0); edge tiles partial) of n masks M (device uint8
 * [n][H][W]) into device fp32 T [n][ceil(H/16)][ceil(W/16)]. */
occl_status occl_cnn_tile_targets(occl_ctx* ctx, const uint8_t* M, int32_t n, int32_t H, int32_t W,
                                  float* T);

/* Exact fallback routed by tile logits (device fp32 [n_views][ceil(H/16)][ceil(W/16)],
 * from occl_cnn_forward or any other source).  A tile with logit
 * z < log(lo / (1 - lo)) (lo = params->cnn_lo, computed in double, rounded to
 * fp32) is written with 0s, one with z > log(hi / (1 - hi)) with 1s, and
 * every other tile with exactly the mask occl_detect writes there.
 * tile_state (device uint8, same shape as the logits, may be NULL) receives
 * 0 / 1 for the filled tiles and 2 for the tiles that took the exact path.
 * The other arguments are those of occl_detect. */
occl_status occl_detect_routed(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                               const double* angles_deg, const float* ratios,
                               const occl_params* params, const float* logits, uint8_t* M,
                               uint8_t* tile_state);

/* The step before the detector: the fused centre disparity D as the
 * pixel-wise median of K per-view disparity maps (Sec. 4 fuses the views'
 * maps by their median).  maps: device fp32 [K][H][W], NaN = no value at that
 * pixel; D: device fp32 [H][W] = median of the non-NaN values (an even count
 * averages the two middle ones, (a + b) * 0.5 in fp32), NaN where all are NaN.
 * K = 1..16 (more: OCCL_ERR_UNSUPPORTED). */
occl_status occl_median_fuse(occl_ctx* ctx, const float* maps, int32_t K, int32_t H, int32_t W,
                             float* D);

/* Ground truth for the quality counts of Eq. (7), by forward warping (a
 * z-buffer).  Under the reading that a centre pixel p lands at p - r*D(p)*u
 * in the view of direction u = (cos alpha, sin alpha), take the nearest target
 * pixel (t = r*D(p), tx = rint(x - t*cos alpha), ty = rint(y - t*sin alpha),
 * fp32, half to even).  M[v][y][x] = 1 iff some pixel (p itself included)
 * lands on the same target with a disparity larger by more than beta.
 * Targets outside the peripheral frame count as well.
 *   D  device fp32 [H][W], finite (non-finite values: OCCL_ERR_INVALID_ARG)
 *   M  device uint8 [n_views][H][W]
 * Reads min/max of D back to size its target grid, so it synchronises. */
occl_status occl_zbuffer(occl_ctx* ctx, const float* D, int32_t H, int32_t W, int32_t n_views,
                         const double* angles_deg, const float* ratios, float beta, uint8_t* M);

/* Waits for the context's stream; reports a pending device error. */
occl_status occl_sync(occl_ctx* ctx);

/* Synchronises, frees every context-owned resource and the context. NULL is a no-op. */
occl_status occl_release(occl_ctx* ctx);

/* Stage timing with HIP events recorded on the context's stream around each
 * stage of every subsequent call (for benchmarks; adds event records
 * between launches).  Enabling resets the accumulators.
 * occl_profile_read synchronises and returns, per stage, the summed
 * milliseconds and the number of launches timed since the last enable. */
#define OCCL_STAGE_EDGES 0      /* k_edges_candidates: Eqs. (1)-(2) + mask clear */
#define OCCL_STAGE_SCANLINES 1  /* k_scanlines: Eqs. (4)-(6) */
#define OCCL_STAGE_CNN 2        /* learned tile proposal (pack, convolutions, routing) */
#define OCCL_STAGE_FALLBACK 3   /* routing: tile states, exact path, confident tiles' fill */
#define OCCL_STAGE_BATCHED 4    /* one graph launch of occl_detect_batched */
#define OCCL_N_STAGES 5
occl_status occl_profile_enable(occl_ctx* ctx, int32_t enable);
occl_status occl_profile_read(occl_ctx* ctx, double* ms /* [OCCL_N_STAGES] */,
                              int64_t* launches /* [OCCL_N_STAGES] */);

/* Measurement of the scanline pass alone: re-enqueues the scanline launches of
 * the context's most recent exact-path frame `reps` times back to back between
 * two HIP events on the context's stream, synchronises, and returns the mean
 * milliseconds per pass (Eqs. (4)-(6), one launch per register class present).
 * The pass only sets mask bytes that the first pass already set, so the masks
 * do not change.  D and M of that call must still be valid (call it right
 * after occl_detect).  OCCL_ERR_STATE when there is no such frame or the
 * context's list workspace has been reallocated since. */
occl_status occl_time_scanlines(occl_ctx* ctx, int32_t reps, double* ms_per_pass);

/* Stage timing of the most recent occl_detect_batched call: its kernels
 * re-enqueued `reps` times outside the graph, on the context's stream (the
 * graph's branches one after the other), with HIP events around each of its
 * two stages; ms (host double[2]) receives the mean milliseconds per batch
 * of each, form (host, may be NULL) which form the batch took:
 *   0  two passes: [0] the edge stage (Eqs. (1)-(2), mask clear, per-frame
 *      prefix), [1] the scanline stage (Eqs. (4)-(6));
 *   1  fused: [0] the mask fill, [1] the fused pass (Eqs. (1)-(6)).
 * The masks are rewritten with the same values.  The frames' D and M must
 * still be valid.  Synchronises.  OCCL_ERR_STATE when there is no such
 * batch or its frame table has been reallocated since. */
occl_status occl_time_batched(occl_ctx* ctx, int32_t reps, double* ms, int32_t* form);

const char* occl_status_string(occl_status s);
const char* occl_last_error(const occl_ctx* ctx);

/* The direction vector the library uses for a baseline angle (host only). */
occl_status occl_direction(double angle_deg, float* c, float* s);

#ifdef __cplusplus
}
#endif

#endif /* OCCL_H */
