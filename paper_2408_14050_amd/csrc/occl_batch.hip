// occl_batch.hip -- many frames of uneven size in one graph launch, and the
// launch-shape autotuner.
//
// A batch is described to the kernels by a table of FrameDesc entries in
// device memory (uploaded from pinned host memory on the context's stream
// before every launch).  The frames are split into two branches of about
// half the pixels each; each branch's edge pass and scanline pass run as
// two persistent kernels (one more per extra scan class present), and the
// branches run side by side.  The graph is captured once (on two private
// capture streams, forked and joined by events) and replayed with
// hipGraphLaunch on the context's stream for every later batch with the same
// signature (table address, frame count, split, launch shape, thresholds and
// views).  Frame pointers and sizes live in the table, not in the graph, so
// new frames of the same shapes reuse the graph.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "occl_ctx.h"
#include "occl_internal.h"

using namespace occl;

namespace {

struct BatchSig {
    int fused;  // 1: clear + fused pass (k_fused), 0: edge and scanline passes
    const void* table;
    int n_frames, total_blocks, n_views, edge_rows, edge_grid, scan_grid;
    int n_branches;
    int cut[kMaxBatchBranches + 1];     // branch b holds frames cut[b] .. cut[b + 1] - 1
    int bstart[kMaxBatchBranches + 1];  // ... and flat edge blocks bstart[b] .. bstart[b + 1] - 1
    unsigned cls_mask[kMaxBatchBranches];
    Thresholds th;
    ViewTable vt;
};

std::vector<uint8_t> sig_bytes(const BatchSig& s) {
    std::vector<uint8_t> b(sizeof(BatchSig));
    std::memcpy(b.data(), &s, sizeof(BatchSig));
    return b;
}

}  // namespace

occl_status occl_ctx::enqueue_batch(int n_frames, const occl_frame* frames, int n_views,
                                    const int* Ls_all, const ViewTable& vt, const Thresholds& th,
                                    const TuneConfig* cfg) {
    size_t px = 0;
    int maxcls = 0;
    for (int f = 0; f < n_frames; ++f) {
        px += (size_t)frames[f].H * frames[f].W;
        for (int v = 0; v < n_views; ++v) maxcls = std::max(maxcls, scan_class(Ls_all[f * n_views + v] / 2));
    }
    const uint64_t bucket = tune_key(true, px, n_views, maxcls);
    TuneConfig tc = cfg ? *cfg : config_for(bucket);
    // edge_rows 0 selects the fused pass where the batch allows it.  Without
    // a measured shape for the bucket, batches of at least 8 tiles per
    // resident block take it.  A block's tile is done when its busiest
    // wavefront is, so a batch of few tiles waits on its tiles with the most
    // candidates, while the two passes spread the candidates over the whole
    // grid: 16 mixed frames (5,642 tiles) 0.32 ms fused against 0.43 ms,
    // 12 frames of 1280x960 (3,600 tiles) 0.29 against 0.28 ms, one such
    // frame 0.11 against 0.05 ms.
    if (!cfg && tuned.find(bucket) == tuned.end()) {
        long long tiles = 0;
        for (int f = 0; f < n_frames; ++f)
            tiles += (long long)((frames[f].W + kEdgeCols - 1) / kEdgeCols) *
                     ((frames[f].H + kFusedTileRows - 1) / kFusedTileRows);
        if (tiles >= 8ll * n_cu * fused_blocks_per_cu()) tc.edge_rows = 0;
    }
    if (tc.edge_rows == 0) {
        if (fusable(n_views, maxcls, th)) return enqueue_batch_fused(n_frames, frames, n_views, Ls_all, vt, th);
        tc.edge_rows = tune_default.edge_rows;
    }
    hipError_t e;
    table_build.assign((size_t)n_frames, FrameDesc{});
    // Branches: consecutive frames of about equal pixel counts, each with its
    // own edge pass and scanline pass, run side by side by the graph (c3,
    // two branches: 1.74-1.79 -> 1.65-1.66 ms; three 1.69 ms, four 1.70-1.73;
    // the second branch's edge pass chained after the first's, to run beside
    // the first's scanline pass, 1.73 ms).  Each branch's blocks are numbered
    // from 0.
    const int nb = std::max(1, std::min(kBatchBranches, n_frames));
    int cut[kMaxBatchBranches + 1] = {};
    cut[nb] = n_frames;
    {
        size_t acc = 0;
        int b = 1;
        for (int f = 0; f < n_frames && b < nb; ++f) {
            acc += (size_t)frames[f].H * frames[f].W;
            while (b < nb && acc * nb >= px * b) cut[b++] = f + 1;
        }
        for (b = 1; b < nb; ++b)  // every branch keeps at least one frame
            cut[b] = std::min(std::max(cut[b], cut[b - 1] + 1), n_frames - (nb - b));
    }
    size_t lists_total = 0;
    int total_blocks = 0;
    int bstart[kMaxBatchBranches + 1] = {};
    unsigned cls_mask[kMaxBatchBranches] = {};
    std::vector<size_t> lists_off(n_frames);
    for (int f = 0, b = 0; f < n_frames; ++f) {
        while (f == cut[b + 1]) bstart[++b] = total_blocks;
        FrameDesc& d = table_build[f];
        describe_frame(&d, frames[f].D, frames[f].M, frames[f].H, frames[f].W, n_views,
                       Ls_all + (size_t)f * n_views, tc.edge_rows);
        d.block_begin = total_blocks - bstart[b];
        total_blocks += d.gx * d.gy;
        lists_off[f] = lists_total;
        lists_total += d.ll.cap * d.ll.copies * n_views;
        for (int ci = 0; ci < kNumClasses; ++ci)
            if (d.cls_start[ci + 1] > d.cls_start[ci]) cls_mask[b] |= 1u << ci;
    }
    bstart[nb] = total_blocks;
    void *lists, *counts, *prefix, *table;
    occl_status s = ensure("blists", std::max<size_t>(lists_total, 1) * sizeof(uint32_t), &lists);
    if (s == OCCL_OK) s = ensure_zeroed("bcounts", (size_t)n_frames * kCountsBytes, &counts);
    if (s == OCCL_OK) s = ensure("bprefix", (size_t)n_frames * kPrefixInts * sizeof(int32_t), &prefix);
    if (s == OCCL_OK) s = ensure("btable", (size_t)n_frames * sizeof(FrameDesc), &table);
    if (s != OCCL_OK) return s;
    for (int f = 0; f < n_frames; ++f) {
        FrameDesc& d = table_build[f];
        d.lists = (uint32_t*)lists + lists_off[f];
        d.counts = (int32_t*)counts + (size_t)f * kCountsInts;
        d.prefix = (int32_t*)prefix + (size_t)f * kPrefixInts;
    }
    s = upload_table(n_frames, table);
    if (s != OCCL_OK) return s;

    BatchSig sg;
    std::memset(&sg, 0, sizeof(sg));
    sg.table = table;
    sg.n_frames = n_frames;
    sg.total_blocks = total_blocks;
    sg.n_views = n_views;
    sg.edge_rows = tc.edge_rows;
    sg.edge_grid = n_cu * edges_batched_blocks_per_cu(tc.edge_rows);
    sg.scan_grid = tc.scan_blocks_per_cu * n_cu;
    sg.n_branches = nb;
    for (int b = 0; b <= nb; ++b) {
        sg.cut[b] = cut[b];
        sg.bstart[b] = bstart[b];
        if (b < nb) sg.cls_mask[b] = cls_mask[b];
    }
    sg.th = th;
    sg.vt = vt;
    const std::vector<uint8_t> key = sig_bytes(sg);
    hipGraphExec_t exec = nullptr;
    for (size_t i = 0; i < graphs.size(); ++i) {
        if (graphs[i].sig == key) {
            exec = graphs[i].exec;
            std::rotate(graphs.begin(), graphs.begin() + i, graphs.begin() + i + 1);
            break;
        }
    }
    if (!exec) {
        if (!cap_stream) {
            e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                cap_stream = nullptr;
                return hip_fail(e, "hipStreamCreate(capture)");
            }
        }
        if (nb > 1 && !cap_fork) {
            e = hipEventCreateWithFlags(&cap_fork, hipEventDisableTiming);
            if (e != hipSuccess) {
                cap_fork = nullptr;
                return hip_fail(e, "hipEventCreate(fork)");
            }
        }
        for (int b = 1; b < nb; ++b) {
            if (!cap_extra[b - 1]) {
                e = hipStreamCreateWithFlags(&cap_extra[b - 1], hipStreamNonBlocking);
                if (e != hipSuccess) {
                    cap_extra[b - 1] = nullptr;
                    return hip_fail(e, "hipStreamCreate(branch)");
                }
            }
            if (!cap_join[b - 1]) {
                e = hipEventCreateWithFlags(&cap_join[b - 1], hipEventDisableTiming);
                if (e != hipSuccess) {
                    cap_join[b - 1] = nullptr;
                    return hip_fail(e, "hipEventCreate(join)");
                }
            }
        }
        e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        // one branch: the edge pass, then the scanline pass of each class present
        auto branch = [&](hipStream_t st, int b) {
            const FrameDesc* t = (const FrameDesc*)table + cut[b];
            const int nf = cut[b + 1] - cut[b], blocks = bstart[b + 1] - bstart[b];
            hipError_t r = launch_edges_batched(st, t, nf, blocks, n_views, vt, th.q_min, tc.edge_rows,
                                                std::min(blocks, sg.edge_grid));
            for (int ci = 0; ci < kNumClasses && r == hipSuccess; ++ci)
                if (cls_mask[b] & (1u << ci)) r = launch_scanlines_batched(st, t, nf, n_views, vt, th, ci, sg.scan_grid);
            return r;
        };
        hipError_t le = hipSuccess;
        if (nb > 1) le = hipEventRecord(cap_fork, cap_stream);
        for (int b = 1; b < nb && le == hipSuccess; ++b) le = hipStreamWaitEvent(cap_extra[b - 1], cap_fork, 0);
        if (le == hipSuccess) le = branch(cap_stream, 0);
        for (int b = 1; b < nb && le == hipSuccess; ++b) {
            le = branch(cap_extra[b - 1], b);
            if (le == hipSuccess) le = hipEventRecord(cap_join[b - 1], cap_extra[b - 1]);
            if (le == hipSuccess) le = hipStreamWaitEvent(cap_stream, cap_join[b - 1], 0);
        }
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cap_stream, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le != hipSuccess ? le : e, "batch capture");
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        GraphEntry g;
        g.sig = key;
        g.graph = graph;
        g.exec = exec;
        graphs.insert(graphs.begin(), std::move(g));
        while (graphs.size() > 4) {
            (void)hipGraphExecDestroy(graphs.back().exec);
            (void)hipGraphDestroy(graphs.back().graph);
            graphs.pop_back();
        }
        ++graph_builds;
    }
    hipEvent_t ev = prof_begin(OCCL_STAGE_BATCHED);
    e = hipGraphLaunch(exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    prof_end(OCCL_STAGE_BATCHED, ev);
    ++graph_launches;
    LastBatch& lb = last_batch;
    lb.valid = true;
    lb.fused = false;
    lb.table = (const FrameDesc*)table;
    lb.n_branches = nb;
    lb.n_views = n_views;
    lb.edge_rows = tc.edge_rows;
    lb.edge_grid = sg.edge_grid;
    lb.scan_grid = sg.scan_grid;
    for (int b = 0; b <= nb; ++b) {
        lb.cut[b] = cut[b];
        lb.bstart[b] = bstart[b];
        if (b < nb) lb.cls_mask[b] = cls_mask[b];
    }
    lb.vt = vt;
    lb.th = th;
    return OCCL_OK;
}

// A repeated batch over the same buffers and shapes has the same frame table:
// its upload (a host-to-device copy between two graph launches, ~28 us of
// idle GPU per launch) is skipped when the device buffer already holds it.
// Stream order keeps that right when the last upload is still queued: every
// later launch runs after it.
occl_status occl_ctx::upload_table(int n, void* dev) {
    const size_t bytes = (size_t)n * sizeof(FrameDesc);
    const uint8_t* src = reinterpret_cast<const uint8_t*>(table_build.data());
    if (dev == table_cached_dev && table_cached.size() == bytes && std::memcmp(table_cached.data(), src, bytes) == 0)
        return OCCL_OK;
    hipError_t e;
    if (!table_host) {
        e = hipHostMalloc((void**)&table_host, kMaxBatch * sizeof(FrameDesc), hipHostMallocDefault);
        if (e != hipSuccess) {
            table_host = nullptr;
            return hip_fail(e, "hipHostMalloc(frame table)");
        }
        e = hipEventCreateWithFlags(&table_event, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    } else {
        e = hipEventSynchronize(table_event);  // the previous upload has left the staging area
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(table)");
    }
    std::memcpy(table_host, src, bytes);
    e = hipMemcpyAsync(dev, table_host, bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(table_event, stream);
    if (e != hipSuccess) {
        table_cached_dev = nullptr;
        return hip_fail(e, "frame table upload");
    }
    table_cached.assign(src, src + bytes);
    table_cached_dev = dev;
    return OCCL_OK;
}

bool occl_ctx::fusable(int n_views, int maxcls, const Thresholds& th) const {
    return maxcls == 0 && n_views >= 1 && n_views <= kFusedMaxViews && th.ns == 1 && !th.bilinear && !th.thin;
}

// The fused form of a batch: one fill kernel clears every mask (and the
// tickets), then one persistent launch runs Eqs. (1)-(6) tile by tile.
occl_status occl_ctx::enqueue_batch_fused(int n_frames, const occl_frame* frames, int n_views, const int* Ls_all,
                                          const ViewTable& vt, const Thresholds& th) {
    hipError_t e;
    table_build.assign((size_t)n_frames, FrameDesc{});
    int total_tiles = 0;
    long long chunks = 0;
    for (int f = 0; f < n_frames; ++f) {
        FrameDesc& d = table_build[f];
        describe_frame(&d, frames[f].D, frames[f].M, frames[f].H, frames[f].W, n_views,
                       Ls_all + (size_t)f * n_views, kFusedTileRows);
        d.block_begin = total_tiles;
        d.lists = nullptr;
        d.counts = nullptr;
        d.prefix = nullptr;
        total_tiles += d.gx * d.gy;
        chunks = std::max<long long>(chunks, ((long long)frames[f].H * frames[f].W * n_views + kClearChunkBytes - 1) /
                                                 kClearChunkBytes);
    }
    void *table, *tickets;
    occl_status s = ensure("btable", (size_t)n_frames * sizeof(FrameDesc), &table);
    if (s == OCCL_OK) s = ensure("ftickets", kFusedTickets * sizeof(uint32_t), &tickets);
    if (s != OCCL_OK) return s;
    s = upload_table(n_frames, table);
    if (s != OCCL_OK) return s;
    const int grid = n_cu * fused_blocks_per_cu();
    const int clear_grid = (int)chunks;  // chunks of the largest frame (grid y: frames)
    BatchSig sg;
    std::memset(&sg, 0, sizeof(sg));
    sg.fused = 1;
    sg.table = table;
    sg.n_frames = n_frames;
    sg.total_blocks = total_tiles;
    sg.n_views = n_views;
    sg.scan_grid = grid;
    sg.edge_grid = clear_grid;
    sg.th = th;
    sg.vt = vt;
    const std::vector<uint8_t> key = sig_bytes(sg);
    hipGraphExec_t exec = nullptr;
    for (size_t i = 0; i < graphs.size(); ++i) {
        if (graphs[i].sig == key) {
            exec = graphs[i].exec;
            std::rotate(graphs.begin(), graphs.begin() + i, graphs.begin() + i + 1);
            break;
        }
    }
    if (!exec) {
        if (!cap_stream) {
            e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                cap_stream = nullptr;
                return hip_fail(e, "hipStreamCreate(capture)");
            }
        }
        e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        const hipError_t le = launch_fused(cap_stream, (const FrameDesc*)table, n_frames, total_tiles, n_views, vt,
                                           th, (unsigned*)tickets, grid, clear_grid);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cap_stream, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le != hipSuccess ? le : e, "batch capture");
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        GraphEntry g;
        g.sig = key;
        g.graph = graph;
        g.exec = exec;
        graphs.insert(graphs.begin(), std::move(g));
        while (graphs.size() > 4) {
            (void)hipGraphExecDestroy(graphs.back().exec);
            (void)hipGraphDestroy(graphs.back().graph);
            graphs.pop_back();
        }
        ++graph_builds;
    }
    hipEvent_t ev = prof_begin(OCCL_STAGE_BATCHED);
    e = hipGraphLaunch(exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    prof_end(OCCL_STAGE_BATCHED, ev);
    ++graph_launches;
    LastBatch& lb = last_batch;
    lb.valid = true;
    lb.fused = true;
    lb.table = (const FrameDesc*)table;
    lb.tickets = (unsigned*)tickets;
    lb.n_branches = 1;
    lb.cut[0] = 0;
    lb.cut[1] = n_frames;
    lb.bstart[0] = 0;
    lb.bstart[1] = total_tiles;
    lb.n_views = n_views;
    lb.edge_grid = clear_grid;
    lb.scan_grid = grid;
    lb.vt = vt;
    lb.th = th;
    return OCCL_OK;
}

// Stage timing of the most recent batch: its kernels re-enqueued eagerly on
// the context's stream (the graph's branches one after the other), `reps`
// times, with HIP events around the edge stage (edge pass + per-frame
// prefix) and the scanline stage of every repetition.  Re-running the
// sequence rewrites the same masks.
extern "C" occl_status occl_time_batched(occl_ctx* ctx, int32_t reps, double* ms, int32_t* form) {
    if (!ctx || !ms || reps < 1) return OCCL_ERR_INVALID_ARG;
    const occl_ctx::LastBatch& lb = ctx->last_batch;
    auto tb = ctx->bufs.find("btable");
    if (!lb.valid || tb == ctx->bufs.end() || tb->second.ptr != (const void*)lb.table)
        return ctx->fail(OCCL_ERR_STATE, "no batch to re-time");
    (void)hipSetDevice(ctx->device);
    hipEvent_t ev[3] = {ctx->take_event(), ctx->take_event(), ctx->take_event()};
    for (hipEvent_t x : ev)
        if (!x) {
            for (hipEvent_t y : ev)
                if (y) ctx->ev_pool.push_back(y);
            return ctx->fail(OCCL_ERR_HIP, "hipEventCreate(time_batched)");
        }
    double acc[2] = {0.0, 0.0};
    hipError_t e = hipSuccess;
    for (int r = 0; r < reps && e == hipSuccess && lb.fused; ++r) {
        // fused form: the mask fill, then the fused pass
        e = hipEventRecord(ev[0], ctx->stream);
        if (e == hipSuccess)
            e = launch_fused_stage(ctx->stream, lb.table, lb.cut[1], lb.bstart[1], lb.n_views, lb.vt, lb.th,
                                   lb.tickets, lb.scan_grid, lb.edge_grid, 0);
        if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
        if (e == hipSuccess)
            e = launch_fused_stage(ctx->stream, lb.table, lb.cut[1], lb.bstart[1], lb.n_views, lb.vt, lb.th,
                                   lb.tickets, lb.scan_grid, lb.edge_grid, 1);
        if (e == hipSuccess) e = hipEventRecord(ev[2], ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
        float t0 = 0.0f, t1 = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t0, ev[0], ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t1, ev[1], ev[2]);
        acc[0] += t0;
        acc[1] += t1;
    }
    for (int r = 0; r < reps && e == hipSuccess && !lb.fused; ++r) {
        e = hipEventRecord(ev[0], ctx->stream);
        for (int b = 0; b < lb.n_branches && e == hipSuccess; ++b) {
            const int nf = lb.cut[b + 1] - lb.cut[b], blocks = lb.bstart[b + 1] - lb.bstart[b];
            e = launch_edges_batched(ctx->stream, lb.table + lb.cut[b], nf, blocks, lb.n_views, lb.vt,
                                     lb.th.q_min, lb.edge_rows, std::min(blocks, lb.edge_grid));
        }
        if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
        for (int b = 0; b < lb.n_branches && e == hipSuccess; ++b)
            for (int ci = 0; ci < kNumClasses && e == hipSuccess; ++ci)
                if (lb.cls_mask[b] & (1u << ci))
                    e = launch_scanlines_batched(ctx->stream, lb.table + lb.cut[b], lb.cut[b + 1] - lb.cut[b],
                                                 lb.n_views, lb.vt, lb.th, ci, lb.scan_grid);
        if (e == hipSuccess) e = hipEventRecord(ev[2], ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
        float t0 = 0.0f, t1 = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t0, ev[0], ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t1, ev[1], ev[2]);
        acc[0] += t0;
        acc[1] += t1;
    }
    for (hipEvent_t x : ev) ctx->ev_pool.push_back(x);
    if (e != hipSuccess) return ctx->hip_fail(e, "time_batched");
    ms[0] = acc[0] / reps;
    ms[1] = acc[1] / reps;
    if (form) *form = lb.fused ? 1 : 0;
    return OCCL_OK;
}

namespace {

// Validation and per-frame scan lengths of a batch call; fills the compacted
// list of non-empty frames and their L values.
occl_status prepare_batch(occl_ctx* ctx, int32_t n_frames, const occl_frame* frames,
                          int32_t n_views, const double* angles_deg, const float* ratios,
                          const occl_params* params, std::vector<occl_frame>* live,
                          std::vector<int>* Ls_all, ViewTable* vt) {
    if (n_frames < 0 || (n_frames > 0 && !frames)) return ctx->fail(OCCL_ERR_INVALID_ARG, "frames");
    occl_status s = ctx->check_params(params, n_views, angles_deg, ratios);
    if (s != OCCL_OK) return s;
    if (params->flags & OCCL_FLAG_USE_CNN) return ctx->fail(OCCL_ERR_UNSUPPORTED, "USE_CNN in a batch");
    if (params->flags & OCCL_FLAG_THIN) return ctx->fail(OCCL_ERR_UNSUPPORTED, "candidate thinning in a batch");
    for (int f = 0; f < n_frames; ++f) {
        const occl_frame& fr = frames[f];
        if (fr.H < 0 || fr.W < 0) return ctx->fail(OCCL_ERR_INVALID_ARG, "negative frame size");
        if (fr.H > 65535 || fr.W > 65535 || (size_t)fr.H * fr.W > ((size_t)1 << 31))
            return ctx->fail(OCCL_ERR_UNSUPPORTED, "frame too large");
        if ((size_t)fr.H * fr.W > 0 && n_views > 0 && (!fr.D || !fr.M))
            return ctx->fail(OCCL_ERR_INVALID_ARG, "frame D or M is NULL");
        if (fr.scan_len_per_view)
            for (int v = 0; v < n_views; ++v)
                if (fr.scan_len_per_view[v] < 1) return ctx->fail(OCCL_ERR_INVALID_ARG, "frame L < 1");
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipSetDevice");
    live->clear();
    Ls_all->clear();
    if (n_views == 0) return OCCL_OK;
    for (int f = 0; f < n_frames; ++f) {
        const occl_frame& fr = frames[f];
        if ((size_t)fr.H * fr.W == 0) continue;
        int Ls[OCCL_MAX_VIEWS];
        s = ctx->resolve_views(fr.D, fr.H, fr.W, n_views, angles_deg, ratios, params,
                               fr.scan_len_per_view, vt, Ls);
        if (s != OCCL_OK) return s;
        live->push_back(fr);
        Ls_all->insert(Ls_all->end(), Ls, Ls + n_views);
    }
    return OCCL_OK;
}

occl_status run_batch(occl_ctx* ctx, const std::vector<occl_frame>& live, const std::vector<int>& Ls,
                      int n_views, const ViewTable& vt, const Thresholds& th, const TuneConfig* cfg) {
    for (size_t f0 = 0; f0 < live.size(); f0 += kMaxBatch) {
        const int n = (int)std::min<size_t>(kMaxBatch, live.size() - f0);
        occl_status s = ctx->enqueue_batch(n, live.data() + f0, n_views, Ls.data() + f0 * n_views, vt,
                                           th, cfg);
        if (s != OCCL_OK) return s;
    }
    return OCCL_OK;
}

}  // namespace

extern "C" occl_status occl_detect_batched(occl_ctx* ctx, int32_t n_frames, const occl_frame* frames,
                                           int32_t n_views, const double* angles_deg,
                                           const float* ratios, const occl_params* params) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    std::vector<occl_frame> live;
    std::vector<int> Ls;
    ViewTable vt{};
    occl_status s = prepare_batch(ctx, n_frames, frames, n_views, angles_deg, ratios, params, &live,
                                  &Ls, &vt);
    if (s != OCCL_OK || live.empty()) return s;
    s = run_batch(ctx, live, Ls, n_views, vt, make_thresholds(params), nullptr);
    if (s != OCCL_OK) return s;
    if (params->flags & OCCL_FLAG_SYNC) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
    }
    return OCCL_OK;
}

// ---------------------------------------------------------------------------
// autotuner: coordinate search over the launch shape, timed with HIP events
// on the context's stream on the caller's own data
// ---------------------------------------------------------------------------
namespace {

const int kEdgeRowsCand[] = {1, 2, 4, 8, 16};
const int kScanBpcCand[] = {2, 4, 8, 16};

template <class F>
occl_status time_config(occl_ctx* ctx, F&& enqueue, int reps, float* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventCreate(tune)");
    occl_status s = OCCL_OK;
    for (int i = 0; i < 2 && s == OCCL_OK; ++i) s = enqueue();
    if (s == OCCL_OK) e = hipEventRecord(a, ctx->stream);
    for (int i = 0; i < reps && s == OCCL_OK && e == hipSuccess; ++i) s = enqueue();
    if (s == OCCL_OK && e == hipSuccess) e = hipEventRecord(b, ctx->stream);
    if (s == OCCL_OK && e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (s == OCCL_OK && e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (s != OCCL_OK) return s;
    if (e != hipSuccess) return ctx->hip_fail(e, "tune timing");
    *ms = t / reps;
    return OCCL_OK;
}

template <class F>
occl_status search(occl_ctx* ctx, F&& enqueue_with, int reps, TuneConfig* best, float* best_ms,
                   bool try_fused = false) {
    *best = ctx->tune_default;
    *best_ms = INFINITY;
    if (try_fused) {
        const TuneConfig c{0, ctx->tune_default.scan_blocks_per_cu};
        float ms;
        occl_status s = time_config(ctx, [&] { return enqueue_with(c); }, reps, &ms);
        if (s != OCCL_OK) return s;
        *best_ms = ms;
        *best = c;
    }
    for (int er : kEdgeRowsCand) {
        TuneConfig c{er, best->scan_blocks_per_cu};
        float ms;
        occl_status s = time_config(ctx, [&] { return enqueue_with(c); }, reps, &ms);
        if (s != OCCL_OK) return s;
        if (ms < *best_ms) {
            *best_ms = ms;
            *best = c;
        }
    }
    for (int bpc : kScanBpcCand) {
        TuneConfig c{best->edge_rows, bpc};
        float ms;
        occl_status s = time_config(ctx, [&] { return enqueue_with(c); }, reps, &ms);
        if (s != OCCL_OK) return s;
        if (ms < *best_ms) {
            *best_ms = ms;
            *best = c;
        }
    }
    return OCCL_OK;
}

}  // namespace

extern "C" occl_status occl_autotune(occl_ctx* ctx, const float* D, int32_t H, int32_t W,
                                     int32_t n_views, const double* angles_deg, const float* ratios,
                                     const occl_params* params, uint8_t* M, int32_t reps,
                                     occl_tune* out) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    occl_status s = ctx->check_params(params, n_views, angles_deg, ratios);
    if (s != OCCL_OK) return s;
    if (H < 1 || W < 1 || n_views < 1 || !D || !M) return ctx->fail(OCCL_ERR_INVALID_ARG, "frame");
    if (H > 65535 || W > 65535 || (size_t)H * W > ((size_t)1 << 31))
        return ctx->fail(OCCL_ERR_UNSUPPORTED, "frame too large");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipSetDevice");
    ViewTable vt{};
    int Ls[OCCL_MAX_VIEWS];
    s = ctx->resolve_views(D, H, W, n_views, angles_deg, ratios, params, nullptr, &vt, Ls);
    if (s != OCCL_OK) return s;
    const Thresholds th = make_thresholds(params);
    TuneConfig best;
    float best_ms;
    s = search(ctx, [&](const TuneConfig& c) { return ctx->enqueue_frame(D, H, W, n_views, Ls, vt, th, M, &c); },
               reps > 0 ? reps : 10, &best, &best_ms);
    if (s != OCCL_OK) return s;
    int maxcls = 0;
    for (int v = 0; v < n_views; ++v) maxcls = std::max(maxcls, scan_class(Ls[v] / 2, th.thin));
    ctx->tuned[tune_key(false, (size_t)H * W, n_views, maxcls)] = best;
    if (out) {
        out->edge_rows = best.edge_rows;
        out->scan_blocks_per_cu = best.scan_blocks_per_cu;
        out->ms = best_ms;
    }
    return OCCL_OK;
}

extern "C" occl_status occl_autotune_batched(occl_ctx* ctx, int32_t n_frames, const occl_frame* frames,
                                             int32_t n_views, const double* angles_deg,
                                             const float* ratios, const occl_params* params,
                                             int32_t reps, occl_tune* out) {
    if (!ctx) return OCCL_ERR_INVALID_ARG;
    std::vector<occl_frame> live;
    std::vector<int> Ls;
    ViewTable vt{};
    occl_status s = prepare_batch(ctx, n_frames, frames, n_views, angles_deg, ratios, params, &live,
                                  &Ls, &vt);
    if (s != OCCL_OK) return s;
    if (live.empty() || (int)live.size() > kMaxBatch)
        return ctx->fail(OCCL_ERR_INVALID_ARG, "autotune needs 1..1024 non-empty frames");
    const Thresholds th = make_thresholds(params);
    TuneConfig best;
    float best_ms;
    size_t px = 0;
    int maxcls = 0;
    for (size_t f = 0; f < live.size(); ++f) {
        px += (size_t)live[f].H * live[f].W;
        for (int v = 0; v < n_views; ++v) maxcls = std::max(maxcls, scan_class(Ls[f * n_views + v] / 2));
    }
    s = search(ctx, [&](const TuneConfig& c) { return run_batch(ctx, live, Ls, n_views, vt, th, &c); },
               reps > 0 ? reps : 5, &best, &best_ms, ctx->fusable(n_views, maxcls, th));
    if (s != OCCL_OK) return s;
    ctx->tuned[tune_key(true, px, n_views, maxcls)] = best;
    if (out) {
        out->edge_rows = best.edge_rows;
        out->scan_blocks_per_cu = best.scan_blocks_per_cu;
        out->ms = best_ms;
    }
    return OCCL_OK;
}

extern "C" occl_status occl_tune_save(const occl_ctx* ctx, const char* path) {
    if (!ctx || !path) return OCCL_ERR_INVALID_ARG;
    FILE* fp = std::fopen(path, "w");
    if (!fp) return OCCL_ERR_INVALID_ARG;
    std::fprintf(fp, "# occl launch shapes: bucket edge_rows scan_blocks_per_cu\n");
    for (const auto& kv : ctx->tuned)
        std::fprintf(fp, "%llu %d %d\n", (unsigned long long)kv.first, kv.second.edge_rows,
                     kv.second.scan_blocks_per_cu);
    const bool ok = std::fclose(fp) == 0;
    return ok ? OCCL_OK : OCCL_ERR_INVALID_ARG;
}

extern "C" occl_status occl_tune_load(occl_ctx* ctx, const char* path) {
    if (!ctx || !path) return OCCL_ERR_INVALID_ARG;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return ctx->fail(OCCL_ERR_INVALID_ARG, "cannot open tune file");
    char line[256];
    std::map<uint64_t, TuneConfig> got;
    while (std::fgets(line, sizeof(line), fp)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        unsigned long long k;
        int er, bpc;
        if (std::sscanf(line, "%llu %d %d", &k, &er, &bpc) != 3 || er < 0 || er > kMaxEdgeRows ||
            (er & (er - 1)) != 0 || bpc < 1 || bpc > 64) {
            std::fclose(fp);
            return ctx->fail(OCCL_ERR_INVALID_ARG, "malformed tune file");
        }
        got[(uint64_t)k] = TuneConfig{er, bpc};
    }
    std::fclose(fp);
    for (const auto& kv : got) ctx->tuned[kv.first] = kv.second;
    return OCCL_OK;
}
