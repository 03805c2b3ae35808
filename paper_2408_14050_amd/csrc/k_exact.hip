// k_exact.hip -- gfx950 kernels of the exact detector (Sec. 3, Eqs. 1-6).
//
// Two launches per frame (plus one per extra register class of long scans);
// the batched forms run every frame of a batch in one launch each and are
// captured together in one graph.
//   edge pass        dense, HBM-bound pass over D (Eqs. 1-2).  One wavefront
//                    per 256-pixel row segment, 4 consecutive pixels per lane
//                    (one float4 of row y and one of row y+1).  The
//                    candidates of every view are compacted with ballots and
//                    appended to the list of their row band with a single
//                    atomic per wavefront.  The same pass writes the zero
//                    background of every mask, so each mask byte costs one
//                    streaming write.  The last block of a frame turns the
//                    segment counters into a class-major prefix for the
//                    scanline pass and clears them for the next frame.
//   scanline pass    one wavefront per candidate scanline (Eqs. 4-6), the
//                    (view, candidate) pairs handed out flat in small groups,
//                    round-robin, so long and short lists balance and all
//                    wavefronts sweep the list (and D) together; for large
//                    frames and for batches each die (XCD) takes its own
//                    eighth of the list so that its L2 holds its part of D.
//                    A scanline of n <= 64*K samples holds K samples per lane.
//                    Ordering by (W, g): W split into maximal non-decreasing
//                    runs; one run is already sorted; up to a few runs are
//                    merged by co-ranks (binary search of every sample in the
//                    other runs); otherwise a bitonic sort whose partners are
//                    reached with DPP and permlane swaps.  The sorted (W, V)
//                    pairs go through LDS for the neighbour test of Eq. (5); hits
//                    are byte stores of 1 into the cleared mask, so
//                    concurrent scanlines need no atomics and the result
//                    does not depend on order.
// The scanline pass has a plain form (N = 1, nearest-pixel sampling, no
// thinning) and a general form with those runtime checks; the host picks the
// plain one whenever a call allows it.
//
// Every fp32 operation that feeds a decision is an explicitly rounded
// intrinsic (__fmul_rn, __fadd_rn, __fsub_rn) and the library is built with
// -ffp-contract=off: no product is ever fused into an add.
#include "occl_internal.h"

namespace occl {
namespace {

// ---------------------------------------------------------------------------
// cross-lane helpers
// ---------------------------------------------------------------------------
#define OCCL_DPP(v, ctrl) ((uint32_t)__builtin_amdgcn_mov_dpp((int)(v), (ctrl), 0xF, 0xF, false))

// Value of lane (lane ^ m) for m in {1, 2, 4, 8, 16, 32}.
//   1, 2  quad permutations
//   4     row_half_mirror then quad reverse:  7 - (i ^ 3) = i ^ 4 within 8
//   8     row_mirror then row_half_mirror:   15 - (i ^ 7) = i ^ 8 within 16
//   16    permlane16_swap (odd rows of one copy <-> even rows of the other)
//   32    permlane32_swap (upper half of one copy <-> lower half of the other)
__device__ __forceinline__ uint32_t xchg(uint32_t v, int m, int lane) {
    switch (m) {
        case 1: return OCCL_DPP(v, 0xB1);
        case 2: return OCCL_DPP(v, 0x4E);
        case 4: return OCCL_DPP(OCCL_DPP(v, 0x141), 0x1B);
        case 8: return OCCL_DPP(OCCL_DPP(v, 0x140), 0x141);
        case 16: {
            const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
            return (lane & 16) ? (uint32_t)p[0] : (uint32_t)p[1];
        }
        default: {
            const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
            return (lane & 32) ? (uint32_t)p[0] : (uint32_t)p[1];
        }
    }
}

__device__ __forceinline__ uint64_t xchg64(uint64_t v, int m, int lane) {
    const uint32_t lo = xchg((uint32_t)v, m, lane);
    const uint32_t hi = xchg((uint32_t)(v >> 32), m, lane);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Loads of D and stores into the masks through global (not flat)
// instructions: the pointers come from the frame table, so the compiler
// cannot infer their address space, and flat accesses also count against
// the LDS wait counter (an LDS wait would then wait for gathers in flight).
__device__ __forceinline__ float ldg(const float* p) {
    return *(const __attribute__((address_space(1))) float*)p;
}
__device__ __forceinline__ float4 ldg4(const float* p) {
    typedef float f4 __attribute__((ext_vector_type(4)));  // float4's copy would take a generic reference
    const f4 v = *(const __attribute__((address_space(1))) f4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stg1(uint8_t* p) {
    *(__attribute__((address_space(1))) uint8_t*)p = 1;
}

// LDS exchange inside one wavefront: keeps the compiler from moving LDS
// accesses across this point (one wavefront's LDS operations are processed
// in order by the hardware).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// fp32 <-> totally ordered uint32 (ascending float order = ascending uint order)
__device__ __forceinline__ uint32_t f2ord(float w) {
    const uint32_t u = __float_as_uint(__fadd_rn(w, 0.0f));  // -0 + 0 = +0: -0 sorts as +0
    return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);  // negative: ~u; else u | sign
}
__device__ __forceinline__ float ord2f(uint32_t o) {
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}

// ---------------------------------------------------------------------------
// Eq. (1) + Eq. (2): edges, candidates, mask clear
// ---------------------------------------------------------------------------
// Exclusive prefix (class-major order) of the frame's segment counters,
// computed once per frame by the last block of the edge pass, which also
// clears the counters for the next frame (so no separate clearing launch is
// needed and the sequence can be replayed from a captured graph).
__device__ void finish_frame(const FrameDesc& f, int n_views) {
    __shared__ int wsum[kMaxEdgeRows];
    const int NT = blockDim.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int C = f.ll.copies;
    const int nseg = n_views * C;
    const int per = (nseg + NT - 1) / NT;
    constexpr int PERMAX = kMaxSegments / 64;
    int c[PERMAX];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < PERMAX; ++j) {
        const int sg = t * per + j;
        c[j] = 0;
        if (j < per && sg < nseg) {
            const int g = f.vord[sg / C] * C + sg % C;
            c[j] = __hip_atomic_load(&f.counts[g * kCounterPad], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        }
        sum += c[j];
    }
    int x = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int run = x - sum;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int j = 0; j < PERMAX; ++j) {
        const int sg = t * per + j;
        if (j < per && sg < nseg) {
            f.prefix[sg] = run;
            const int g = f.vord[sg / C] * C + sg % C;
            __hip_atomic_store(&f.counts[g * kCounterPad], 0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        run += c[j];
    }
    if (t == NT - 1) f.prefix[nseg] = run;
}

// One edge-pass block (bx, by) of frame f: blockDim.x / 64 wavefronts on
// consecutive rows.  E > gamma is decided without a square root:
// q = E_x^2 + E_y^2 (fp32, same rounding as the definition) is compared with
// q_min, the smallest fp32 q whose correctly rounded square root exceeds
// gamma (computed on the host), which is exactly sqrt_rn(q) > gamma.
constexpr int kViewChunk = 8;

// This lane's D values of edge-pass block (bx, by) of frame f: row y at
// x0 .. x0 + 4 and row y + 1 at x0 .. x0 + 3 (0 outside the frame).
struct EdgeIn {
    float d0[4], d1[4], dn;
};

__device__ __forceinline__ bool edge_vec(const FrameDesc& f) {
    return ((f.W & 3) == 0) && ((reinterpret_cast<uintptr_t>(f.D) & 15) == 0) &&
           ((reinterpret_cast<uintptr_t>(f.M) & 3) == 0);
}

__device__ __forceinline__ EdgeIn edge_load(const FrameDesc& f, int bx, int by) {
    const int H = f.H, W = f.W;
    const int y = by * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    const int x0 = bx * kEdgeCols + (int)(threadIdx.x & 63) * 4;
    EdgeIn in{{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, 0.0f};
    if (y < H && x0 < W) {
        const float* row = f.D + (size_t)y * W;
        const bool next_row = (y + 1 < H);
        if (edge_vec(f)) {  // W % 4 == 0 and D 16-byte aligned, so x0 + 3 < W
            const float4 a = ldg4(row + x0);
            in.d0[0] = a.x; in.d0[1] = a.y; in.d0[2] = a.z; in.d0[3] = a.w;
            if (next_row) {
                const float4 b = ldg4(row + W + x0);
                in.d1[0] = b.x; in.d1[1] = b.y; in.d1[2] = b.z; in.d1[3] = b.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool inside = (x0 + j < W);
                in.d0[j] = inside ? ldg(row + x0 + j) : 0.0f;
                in.d1[j] = (inside && next_row) ? ldg(row + W + x0 + j) : 0.0f;
            }
        }
        in.dn = (x0 + 4 < W) ? ldg(row + x0 + 4) : 0.0f;
    }
    return in;
}

template <bool kFinish>
__device__ void edge_block(const FrameDesc& f, int bx, int by, int n_views, const ViewTable& vt,
                           float q_min, const EdgeIn& in) {
    const int H = f.H, W = f.W;
    const int lane = threadIdx.x & 63;
    const int rows = blockDim.x >> 6;
    const int y = by * rows + (threadIdx.x >> 6);
    const int x0 = bx * kEdgeCols + lane * 4;
    const bool vec = edge_vec(f);
    const bool row_ok = (y < H);
    const bool live = row_ok && x0 < W;
    if (row_ok) {
        const bool next_row = (y + 1 < H);
        const float* d0 = in.d0;
        const float* d1 = in.d1;
        const float dn = in.dn;
        float ex[4], ey[4];
        bool strong[4];
        bool any = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + j;
            const float right = (j < 3) ? d0[j + 1] : dn;
            ex[j] = (x + 1 < W) ? __fsub_rn(right, d0[j]) : 0.0f;
            ey[j] = next_row ? __fsub_rn(d1[j], d0[j]) : 0.0f;
            const float q = __fadd_rn(__fmul_rn(ex[j], ex[j]), __fmul_rn(ey[j], ey[j]));
            strong[j] = live && (x < W) && (q >= q_min);
            any |= strong[j];
        }
        // Every mask byte of the segment starts at 0.  The stores are issued
        // while the list reservation's atomic is in flight.
        auto clear_mask = [&]() {
            if (!live) return;
            const size_t HW = (size_t)H * W;
            for (int v = 0; v < n_views; ++v) {
                uint8_t* mrow = f.M + v * HW + (size_t)y * W;
                if (vec) {
                    *reinterpret_cast<uint32_t*>(mrow + x0) = 0u;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (x0 + j < W) mrow[x0 + j] = 0;
                }
            }
        };
        bool cleared = false;  // uniform
        if (__ballot(any)) {
            const int band = by / f.ll.block_rows_per_copy;
            const uint32_t pix = ((uint32_t)y << 16) | (uint32_t)x0;  // packed (y, x); W, H <= 65535
            // Views go in chunks of kViewChunk: the candidate bits of every view
            // of the chunk first, then one atomic instruction in which lane i
            // reserves view v0 + i's entries (a single round trip for the
            // chunk), then the appends.
            for (int v0 = 0; v0 < n_views; v0 += kViewChunk) {
                uint32_t m4all = 0;  // bit 4 i + j: pixel x0 + j is a candidate of view v0 + i
                int tot[kViewChunk], off[kViewChunk];
#pragma unroll
                for (int i = 0; i < kViewChunk; ++i) {
                    tot[i] = 0;
                    off[i] = 0;
                    const int v = v0 + i;
                    if (v >= n_views) continue;  // uniform
                    const float c = vt.c[v], s = vt.s[v];
                    uint64_t b[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float dot = __fadd_rn(__fmul_rn(ex[j], c), __fmul_rn(ey[j], s));
                        const bool cand = strong[j] && (dot > 0.0f);
                        m4all |= cand ? (1u << (4 * i + j)) : 0u;
                        b[j] = __ballot(cand);
                    }
                    tot[i] = __popcll(b[0]) + __popcll(b[1]) + __popcll(b[2]) + __popcll(b[3]);
                    off[i] = (int)(lanes_below(b[0]) + lanes_below(b[1]) + lanes_below(b[2]) +
                                   lanes_below(b[3]));
                }
                int my_tot = 0;
#pragma unroll
                for (int i = 0; i < kViewChunk; ++i) my_tot = (lane == i) ? tot[i] : my_tot;
                int my_base = 0;
                if (my_tot > 0)
                    my_base = atomicAdd(&f.counts[((v0 + lane) * f.ll.copies + band) * kCounterPad], my_tot);
                if (!cleared) {
                    clear_mask();
                    cleared = true;
                }
                // every base into a scalar before the first append (the appends'
                // stores would otherwise sit between the atomic and its reads)
                int bs[kViewChunk];
#pragma unroll
                for (int i = 0; i < kViewChunk; ++i) bs[i] = __builtin_amdgcn_readlane(my_base, i);
#pragma unroll
                for (int i = 0; i < kViewChunk; ++i) {
                    if (tot[i] == 0) continue;
                    const int seg = (v0 + i) * f.ll.copies + band;
                    uint32_t* dst = f.lists + (size_t)seg * f.ll.cap + bs[i] + off[i];
                    const uint32_t m4 = m4all >> (4 * i);
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (m4 & (1u << j)) *dst++ = pix + j;
                }
            }
        }
        if (!cleared) clear_mask();
    }
    if constexpr (!kFinish) return;  // the batched path finishes frames in k_finish_frames
    // The last block of the frame turns the counters into the frame's prefix.
    // Completion is counted in two levels (kDoneGroups group counters, then
    // one top counter) so no single address takes one atomic per block.  No
    // fence is needed: every segment atomic of this block has returned (its
    // result addressed the list stores) before the completion atomic,
    // device-scope atomics are performed at the coherence point, the last
    // block reads the counters with atomic loads, and the list entries are
    // only read by the next launch.
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* done = reinterpret_cast<unsigned*>(f.counts + kMaxSegments * kCounterPad);
        const unsigned gy = f.gy;
        const unsigned grp = by % kDoneGroups;
        const unsigned groups = gy < (unsigned)kDoneGroups ? gy : (unsigned)kDoneGroups;
        const unsigned in_grp = f.gx * ((gy - grp + kDoneGroups - 1) / kDoneGroups);
        int last = 0;
        if (atomicAdd(&done[(1 + grp) * kCounterPad], 1u) == in_grp - 1)
            last = (atomicAdd(&done[0], 1u) == groups - 1) ? 1 : 0;
        s_last = last;
    }
    __syncthreads();
    if (s_last) {
        finish_frame(f, n_views);
        unsigned* done = reinterpret_cast<unsigned*>(f.counts + kMaxSegments * kCounterPad);
        for (int i = threadIdx.x; i <= kDoneGroups; i += blockDim.x)
            __hip_atomic_store(&done[i * kCounterPad], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// Held to 8 wavefronts per SIMD like the scanline pass: with frames in flight
// the next frame's edge blocks then share the CUs with the current frame's
// scanline blocks more readily (c1, three frames in flight: 18.0-19.1 ->
// 17.0 us per frame).
__global__ __launch_bounds__(64 * kMaxEdgeRows, 8) void k_edges(FrameDesc f, int n_views, ViewTable vt,
                                                               float q_min) {
    edge_block<true>(f, blockIdx.x, blockIdx.y, n_views, vt, q_min, edge_load(f, blockIdx.x, blockIdx.y));
}

// Every frame of a batch: a persistent grid walks the flat list of edge-pass
// blocks of all frames (frame fi owns [block_begin, next block_begin)).
__global__ __launch_bounds__(64 * kMaxEdgeRows, 8) void k_edges_batched(
    const FrameDesc* __restrict__ table, int n_frames, int total_blocks, int n_views, ViewTable vt,
    float q_min) {
    // the frames' first blocks, staged once so that locating a virtual block's
    // frame is an LDS search rather than a chain of dependent global loads
    __shared__ int begin[kMaxBatch];
    for (int i = threadIdx.x; i < n_frames; i += blockDim.x) begin[i] = table[i].block_begin;
    __syncthreads();
    // Software-pipelined: the loads of the block's next virtual block are
    // issued before this one's list reservation, so the load and atomic round
    // trips overlap.  Held to 8 wavefronts per SIMD (a few bytes of spills):
    // the persistent grid is sized to what is resident (64 mixed frames:
    // 2.31 -> 2.26 ms).
    auto frame_of = [&](int vb, int from) {  // last frame with block_begin <= vb
        int lo = from, hi = n_frames - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (begin[mid] <= vb) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    int vb = blockIdx.x;
    if (vb >= total_blocks) return;
    int fi = frame_of(vb, 0);
    int local = vb - begin[fi];
    EdgeIn cur = edge_load(table[fi], local % table[fi].gx, local / table[fi].gx);
    while (vb < total_blocks) {
        const int nvb = vb + gridDim.x;
        int nfi = fi, nlocal = 0;
        EdgeIn nxt{};
        if (nvb < total_blocks) {
            nfi = frame_of(nvb, fi);
            nlocal = nvb - begin[nfi];
            nxt = edge_load(table[nfi], nlocal % table[nfi].gx, nlocal / table[nfi].gx);
        }
        const FrameDesc& f = table[fi];
        edge_block<false>(f, local % f.gx, local / f.gx, n_views, vt, q_min, cur);
        vb = nvb;
        fi = nfi;
        local = nlocal;
        cur = nxt;
    }
}

// After the batched edge pass: one block per frame turns its segment counters
// into the frame's prefix and clears them (what the frame's last edge block
// does on the single-frame path).
__global__ __launch_bounds__(256) void k_finish_frames(const FrameDesc* __restrict__ table, int n_views) {
    finish_frame(table[blockIdx.x], n_views);
}

// ---------------------------------------------------------------------------
// Eq. (4) - Eq. (6): one scanline per wavefront
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void cmp_swap_stage(uint64_t (&key)[K], int size, int stride, int lane) {
    if (stride >= 64) {
        const int ks = stride >> 6;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if ((k & ks) == 0) {
                const int kp = k | ks;
                const bool up = (((k * 64 + lane) & size) == 0);
                const uint64_t a = key[k], b = key[kp];
                const bool sw = up ? (a > b) : (a < b);
                key[k] = sw ? b : a;
                key[kp] = sw ? a : b;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t o = xchg64(key[k], stride, lane);
            const bool up = (((k * 64 + lane) & size) == 0);
            const bool lower = ((lane & stride) == 0);
            const bool lt = key[k] < o;
            const uint64_t mn = lt ? key[k] : o;
            const uint64_t mx = lt ? o : key[k];
            key[k] = (lower == up) ? mn : mx;
        }
    }
}

template <int K>
constexpr int log2_keys() { return K == 1 ? 6 : K == 2 ? 7 : K == 4 ? 8 : K == 8 ? 9 : 10; }

// Ascending bitonic sort of 64*K keys; element e = k*64 + lane lives in key[k].
template <int K>
__device__ __forceinline__ void bitonic_sort(uint64_t (&key)[K], int lane) {
    constexpr int LG = log2_keys<K>();
#pragma unroll
    for (int ls = 1; ls <= LG; ++ls) {
#pragma unroll
        for (int lt = ls - 1; lt >= 0; --lt) cmp_swap_stage<K>(key, 1 << ls, 1 << lt, lane);
    }
}

// Ascending sort of the 64*K keys of key[]: the bitonic network for a power
// of two K, else over the next power of two with the added slots holding
// ~0 (above every key), so the sorted keys fill slots 0 .. K - 1 again.
template <int K>
__device__ __forceinline__ void sort_keys(uint64_t (&key)[K], int lane) {
    if constexpr ((K & (K - 1)) == 0) {
        bitonic_sort<K>(key, lane);
    } else {
        constexpr int KP = K < 4 ? 4 : (K < 8 ? 8 : 16);
        uint64_t kp[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) kp[k] = k < K ? key[k] : ~0ull;
        bitonic_sort<KP>(kp, lane);
#pragma unroll
        for (int k = 0; k < K; ++k) key[k] = kp[k];
    }
}

struct WaveLds {
    float2* WVin;   // (W, V) by offset index e (W NaN where the sample is dropped)
    uint32_t* Oin;  // f2ord(W) by e (the search keys of the co-rank merge)
    float2* WVs;    // (W, V) in sorted order (merge and sort paths)
    int* rs;        // run starts (co-rank path), kMaxRunsCap + 1 entries
};

constexpr int kMaxRunsCap = 16;

// Largest number of monotone runs for which the co-rank path is used
// (above it the full sort is cheaper).
template <int K>
constexpr int max_runs() { return K == 1 ? 4 : K == 2 ? 5 : K <= 4 ? 6 : K <= 8 ? 8 : 12; }

// (W, e) ordering of two samples: a before b
__device__ __forceinline__ bool key_less(float wa, int ea, float wb, int eb) {
    return wa < wb || (wa == wb && ea < eb);
}

// G (all scanline forms): 1 when the call may use the bilinear sampling
// variant, thinning or more than one neighbour per side (runtime checks), 0 for the plain exact path with N = 1, where those checks
// are compiled out (fewer registers: c2 pass 2.93 -> 2.64 ms, c1 25.8 ->
// 25.3 us).
template <int K, int G>
__device__ __forceinline__ void mark_hit(uint8_t* __restrict__ Mv, int W, int cx, int cy, float c,
                                         float s, int g) {
    const float gf = (float)g;
    const int ix = (int)rintf(__fadd_rn((float)cx, __fmul_rn(c, gf)));
    const int iy = (int)rintf(__fadd_rn((float)cy, __fmul_rn(s, gf)));
    Mv[(size_t)iy * W + ix] = 1;
}

// Eq. (2) at the pixel of scanline offset g (Eq. (4) rounding), with the
// edge pass's arithmetic: false outside the frame.
__device__ __forceinline__ bool candidate_at(const float* __restrict__ D, int H, int W, int cx, int cy,
                                             float c, float s, int g, float q_min) {
    const float gf = (float)g;
    const int ix = (int)rintf(__fadd_rn((float)cx, __fmul_rn(c, gf)));
    const int iy = (int)rintf(__fadd_rn((float)cy, __fmul_rn(s, gf)));
    if ((uint32_t)ix >= (uint32_t)W || (uint32_t)iy >= (uint32_t)H) return false;
    const size_t o = (size_t)iy * W + ix;
    const float d = D[o];
    const float ex = (ix + 1 < W) ? __fsub_rn(D[o + 1], d) : 0.0f;
    const float ey = (iy + 1 < H) ? __fsub_rn(D[o + W], d) : 0.0f;
    const float q = __fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey));
    const float dot = __fadd_rn(__fmul_rn(ex, c), __fmul_rn(ey, s));
    return (q >= q_min) && (dot > 0.0f);
}

// Candidate thinning (variant): the number of samples of the candidate's
// merged window, or 0 for a follower.  A candidate whose pixel at g = -1 is
// itself a candidate is a follower (its scanline is covered by the head of
// its run); any other candidate scans g = -h .. h + m over the run of m <= h
// candidates at g = 1, 2, ...  Lane t of a 64-offset chunk tests offset t
// (t = 0 stands for g = -1); the run is the trailing ones of the ballots.
__device__ __forceinline__ int thin_window(const float* __restrict__ D, int H, int W, int cx, int cy, float c,
                                           float s, int h, float q_min, int lane) {
    int m = 0;
    for (int t0 = 0; t0 <= h; t0 += 64) {
        const int t = t0 + lane;
        const bool is_c = (t <= h) && candidate_at(D, H, W, cx, cy, c, s, t == 0 ? -1 : t, q_min);
        uint64_t b = __ballot(is_c);
        if (t0 == 0) {
            if (b & 1ull) return 0;  // follower
            b |= 1ull;               // the candidate itself opens the run
        }
        const uint64_t gap = ~b;
        if (gap == 0) {
            m += (t0 == 0) ? 63 : 64;
            continue;
        }
        m += (__ffsll((unsigned long long)gap) - 1) - (t0 == 0 ? 1 : 0);
        break;
    }
    return 2 * h + 1 + m;  // offsets t > h are never candidates, so m <= h
}

template <int K, int G>
__device__ __forceinline__ void order_test_lds(uint8_t* __restrict__ Mv, int W, int cx, int cy,
                                               float c, float s, int h, const Thresholds& th,
                                               const WaveLds& L, int lane, const float (&wk)[K],
                                               const float (&vk)[K], const uint64_t (&vmask)[K],
                                               const bool (&kept)[K], const uint32_t (&pofs)[K]);

// One scanline: the n <= 64 K samples of offsets g = -h .. n - 1 - h
// (n = 2h + 1, or a thinning head's merged window).
template <int K, int G>
__device__ __forceinline__ void scanline(const float* __restrict__ D, int H, int W,
                                         uint8_t* __restrict__ Mv, int cx, int cy, float c,
                                         float s, float r, int h, int n, const Thresholds& th,
                                         const WaveLds& L, int lane) {
    float wk[K], vk[K];  // this lane's W and V of slot k
    uint64_t vmask[K];
    bool kept[K];  // this lane's sample of slot k is in the frame (the bit of vmask[k])
    uint32_t pofs[K];  // pixel offset iy * W + ix of each kept sample (H * W < 2^32)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // branch-free: the gather address is clamped into the frame and the
        // value of a dropped sample is discarded
        const int e = k * 64 + lane;
        const float gf = (float)(e - h);
        const float px = __fadd_rn((float)cx, __fmul_rn(c, gf));
        const float py = __fadd_rn((float)cy, __fmul_rn(s, gf));
        const int ix = (int)rintf(px);
        const int iy = (int)rintf(py);
        const bool valid = (e < n) & ((uint32_t)ix < (uint32_t)W) & ((uint32_t)iy < (uint32_t)H);
        const uint32_t po = (uint32_t)iy * (uint32_t)W + (uint32_t)ix;  // H * W < 2^32
        float Vr;
        if (G && th.bilinear) {  // variant: bilinear V at (px, py), taps clamped into the frame
            const float fx0 = floorf(px), fy0 = floorf(py);
            const float fx = __fsub_rn(px, fx0), fy = __fsub_rn(py, fy0);
            const int x0 = (int)fx0, y0 = (int)fy0;
            const int xa = min(max(x0, 0), W - 1), xb = min(max(x0 + 1, 0), W - 1);
            const int ya = min(max(y0, 0), H - 1), yb = min(max(y0 + 1, 0), H - 1);
            const float a = D[(size_t)ya * W + xa], b = D[(size_t)ya * W + xb];
            const float cc = D[(size_t)yb * W + xa], d = D[(size_t)yb * W + xb];
            const float gx = __fsub_rn(1.0f, fx), gy = __fsub_rn(1.0f, fy);
            const float top = __fadd_rn(__fmul_rn(gx, a), __fmul_rn(fx, b));
            const float bot = __fadd_rn(__fmul_rn(gx, cc), __fmul_rn(fx, d));
            Vr = __fadd_rn(__fmul_rn(gy, top), __fmul_rn(fy, bot));
        } else {
            Vr = ldg(D + (valid ? po : 0u));  // a dropped sample reads pixel 0 and is discarded
        }
        pofs[k] = po;  // used for kept samples only
        const float V = valid ? Vr : 0.0f;
        const float w = valid ? __fsub_rn(gf, __fmul_rn(r, Vr)) : __int_as_float(0x7fc00000);
        L.WVin[e] = make_float2(w, V);  // W NaN: dropped
        L.Oin[e] = f2ord(w);
        wk[k] = w;
        vk[k] = V;
        vmask[k] = __ballot(valid);
        kept[k] = valid;
    }
    wave_lds_sync();
    order_test_lds<K, G>(Mv, W, cx, cy, c, s, h, th, L, lane, wk, vk, vmask, kept, pofs);
}

// Ordering (Eq. (4)'s sort) and Eqs. (5)-(6) of one scanline whose samples
// sit in registers (wk, vk, kept, pofs, vmask of slot k = offsets k*64 +
// lane) and, by offset, in L.WVin / L.Oin.
template <int K, int G>
__device__ __forceinline__ void order_test_lds(uint8_t* __restrict__ Mv, int W, int cx, int cy,
                                               float c, float s, int h, const Thresholds& th,
                                               const WaveLds& L, int lane, const float (&wk)[K],
                                               const float (&vk)[K], const uint64_t (&vmask)[K],
                                               const bool (&kept)[K], const uint32_t (&pofs)[K]) {
    constexpr int N = 64 * K;
    // descents W_e < W_{e-1} (both kept; NaN compares false): they split the
    // kept samples into maximal runs of non-decreasing W
    uint64_t dm[K];
    int nvalid = 0, e_lo = -1, ndesc = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = k * 64 + lane;
        const float wp = (e > 0) ? L.WVin[e - 1].x : __int_as_float(0x7fc00000);
        dm[k] = __ballot(wk[k] < wp);
        ndesc += __popcll(dm[k]);
        nvalid += __popcll(vmask[k]);
        if (vmask[k] && e_lo < 0) e_lo = k * 64 + __ffsll((unsigned long long)vmask[k]) - 1;
    }
    if (nvalid == 0) return;
    const int e_hi = e_lo + nvalid - 1;  // the kept offsets are one contiguous run
    const int R = ndesc + 1;

    // sorted position of every kept sample (pk) and the sorted pairs WVs
    int pk[K];
    const float2* WVs;
    if (R == 1) {
        // already in (W, g) order: sorted position p is offset e_lo + p
#pragma unroll
        for (int k = 0; k < K; ++k) pk[k] = k * 64 + lane - e_lo;
        WVs = L.WVin + e_lo;
    } else if (R <= max_runs<K>()) {
        // ---- co-rank merge: every run is sorted by (W, e); the sorted position
        // of sample e is its index in its own run plus, for every other run,
        // the number of that run's keys below (W_e, e) (binary search) ----
        int before = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if ((dm[k] >> lane) & 1ull) L.rs[1 + before + (int)lanes_below(dm[k])] = k * 64 + lane;
            before += __popcll(dm[k]);
        }
        if (lane == 0) {
            L.rs[0] = e_lo;
            L.rs[R] = e_hi + 1;
        }
        wave_lds_sync();
        // longest run of the scanline bounds the search
        int mmax = 1;
        for (int rr = 0; rr < R; ++rr) mmax = max(mmax, L.rs[rr + 1] - L.rs[rr]);
        const int top = 31 - __clz(mmax);
        int e_[K], own_[K], pos_[K];
        uint32_t oe_[K];
        before = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e0 = k * 64 + lane;
            const bool valid = kept[k];
            e_[k] = valid ? e0 : e_lo;  // dropped lanes ride on a kept sample
            // run index: descents at offsets <= e (below this lane, and its own)
            own_[k] = valid ? before + (int)lanes_below(dm[k]) + (int)((dm[k] >> lane) & 1ull) : 0;
            before += __popcll(dm[k]);
            oe_[k] = f2ord(wk[k]);
            pos_[k] = e_[k] - L.rs[own_[k]];
        }
        // The searches of up to KC samples of a lane advance in lockstep, so
        // their dependent LDS reads overlap instead of queueing one after
        // the other (K = 6: all six, 3840x2160 x15 frame 1.96 -> 1.90 ms
        // against three; two were slower).
        constexpr int KC = K <= 6 ? K : 4;  // divides K
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += KC) {
            for (int i = 0; i + 1 < R; ++i) {
                uint32_t T[KC];
                int s0[KC], base[KC], len[KC];
#pragma unroll
                for (int j = 0; j < KC; ++j) {
                    const int own = own_[k0 + j];
                    const int rr = i < own ? i : i + 1;
                    // keys of run rr below (W_e, e): O_j < ord(W_e), or <= for
                    // a run before e (equal W precede e); branch-free lower bound
                    T[j] = oe_[k0 + j] + (rr < own ? 1u : 0u);
                    s0[j] = L.rs[rr];
                    base[j] = s0[j];
                    len[j] = L.rs[rr + 1] - s0[j];
                }
                for (int st = top; st >= 0; --st) {
#pragma unroll
                    for (int j = 0; j < KC; ++j) {
                        const int half = len[j] >> 1;
                        base[j] = (L.Oin[base[j] + half] < T[j]) ? base[j] + half : base[j];
                        len[j] -= half;
                    }
                }
#pragma unroll
                for (int j = 0; j < KC; ++j)
                    pos_[k0 + j] += base[j] - s0[j] + ((L.Oin[base[j]] < T[j]) ? 1 : 0);
            }
        }
        // a kept sample writes its own (W, V) (registers) at its sorted
        // position; nothing reads WVin any more (WVs may share its storage)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            pk[k] = pos_[k];
            if (kept[k]) {
                L.WVs[pos_[k]] = make_float2(wk[k], vk[k]);
            }
        }
        WVs = L.WVs;
        wave_lds_sync();
    } else {
        // ---- many runs: bitonic sort of (W, e) keys ----
        uint64_t key[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t e = (uint32_t)(k * 64 + lane);
            key[k] = kept[k] ? (((uint64_t)f2ord(wk[k]) << 32) | e) : ~0ull;
        }
        sort_keys<K>(key, lane);
        // the sorted array holds the origin of position p in key[k]; scatter the
        // inverse (origin -> position) into the key array, unused on this
        // path, so the test below runs per kept sample.  Every read of WVin
        // comes before the first write (WVs may share WVin's storage).
        float vv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vv[k] = L.WVin[(k * 64 + lane < nvalid) ? (uint32_t)key[k] : 0u].y;
        int* inv = reinterpret_cast<int*>(L.Oin);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int p = k * 64 + lane;
            if (p < nvalid) {
                const uint32_t o = (uint32_t)key[k];
                L.WVs[p] = make_float2(ord2f((uint32_t)(key[k] >> 32)), vv[k]);
                inv[o] = p;
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int k = 0; k < K; ++k) pk[k] = inv[min(k * 64 + lane, N - 1)];
        WVs = L.WVs;
        wave_lds_sync();
    }
    // Eq. (5) at every kept sample's sorted position, Eq. (6) at its pixel
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = k * 64 + lane;
        const bool valid = kept[k];
        const int p = valid ? pk[k] : 0;
        // every route wrote this sample's own W and V at its sorted position p
        const float Wp = wk[k];
        const float Vp = vk[k];
        bool hit = false;
        const int ns = G ? th.ns : 1;  // the plain form serves N = 1 only
        for (int d = 1; d <= ns; ++d) {
            const int jl = max(p - d, 0), jr = min(p + d, nvalid - 1);
            const float2 nl = WVs[jl], nr = WVs[jr];
            const float wl = nl.x, vl = nl.y, wr = nr.x, vr = nr.y;
            hit |= (p - d >= 0) & (fabsf(__fsub_rn(Wp, wl)) < th.zeta) & (__fsub_rn(vl, Vp) > th.beta);
            hit |= (p + d < nvalid) & (fabsf(__fsub_rn(Wp, wr)) < th.zeta) &
                   (__fsub_rn(vr, Vp) > th.beta);
        }
        if (valid & hit) {
            if constexpr (G)
                mark_hit<K, G>(Mv, W, cx, cy, c, s, e - h);
            else
                stg1(Mv + pofs[k]);  // the pixel the gather read
        }
    }
    wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Plain form (N = 1, nearest-pixel V, no thinning) of the scanlines of
// at most 128 samples: the samples and the one-run test of Eq. (5) stay in
// registers (neighbours through DPP); two runs take their sorted neighbours
// from a binary search over the other run in LDS; three or more runs go
// through the general LDS ordering.
// ---------------------------------------------------------------------------
// Wave-wide shift by one lane (DPP wave_shr:1 / wave_shl:1): lane i receives
// v of lane i - 1 (up) or i + 1 (down); the lane that has no source lane
// keeps `fill`.
__device__ __forceinline__ float wave_up1(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), 0x138, 0xF, 0xF,
                                                      false));
}
__device__ __forceinline__ float wave_down1(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), 0x130, 0xF, 0xF,
                                                      false));
}
// Eq. (5) with one neighbour per side and Eq. (6) for sorted positions q =
// 64 k + lane holding (W, V) of the sample whose pixel offset is po; W NaN
// marks a position without a sample.
template <int K>
__device__ __forceinline__ void test_sorted(uint8_t* __restrict__ Mv, const float (&w)[K], const float (&v)[K],
                                            const uint32_t (&po)[K], const Thresholds& th) {
    const float NaN = __int_as_float(0x7fc00000);
    auto lanef = [](float x, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); };
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int kp = k > 0 ? k - 1 : 0, kn = k + 1 < K ? k + 1 : k;
        // neighbours across the slot boundary: lane 63 of slot k - 1, lane 0 of slot k + 1
        const float wl = wave_up1(w[k], k > 0 ? lanef(w[kp], 63) : NaN);
        const float vl = wave_up1(v[k], k > 0 ? lanef(v[kp], 63) : 0.0f);
        const float wr = wave_down1(w[k], k + 1 < K ? lanef(w[kn], 0) : NaN);
        const float vr = wave_down1(v[k], k + 1 < K ? lanef(v[kn], 0) : 0.0f);
        const bool hit = ((fabsf(__fsub_rn(w[k], wl)) < th.zeta) & (__fsub_rn(vl, v[k]) > th.beta)) |
                         ((fabsf(__fsub_rn(w[k], wr)) < th.zeta) & (__fsub_rn(vr, v[k]) > th.beta));
        if (hit) stg1(Mv + po[k]);  // a NaN W (no sample here) never hits
    }
}

// Two runs A = [e_lo, j0) and B = [j0, e_hi] (each non-decreasing in W; e_lo
// < j0 <= e_hi): the sorted order of (W, e) interleaves them, so the sorted
// predecessor of a sample is the later of its predecessor in its own run and
// the last sample of the other run before it, and its successor is the
// earlier of its successor in its own run and the first sample of the other
// run after it.  That rank in the other run comes from a binary search over
// the other run's ord(W) keys (a sample of A precedes a sample of B of equal
// W, as its offset is smaller), so neither a sorted array nor a merge is
// built.  Then Eq. (5) with one neighbour per side and Eq. (6).
// LDS: WVin holds (W, V) by offset; WVs holds the keys of A and of B from
// index 0 each, padded with ~0 (above every key), 2 N words.
template <int K>
__device__ __forceinline__ void two_runs(uint8_t* __restrict__ Mv, const float (&wk)[K], const float (&vk)[K],
                                         const bool (&kept)[K], const uint32_t (&pofs)[K], int e_lo, int j0,
                                         int e_hi, const Thresholds& th, const WaveLds& L, int lane) {
    constexpr int N = 64 * K;
    uint32_t* OA = reinterpret_cast<uint32_t*>(L.WVs);
    uint32_t* OB = OA + N;
    const int lenA = j0 - e_lo, lenB = e_hi - j0 + 1;
    uint32_t key[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = k * 64 + lane;
        OA[e] = ~0u;
        OB[e] = ~0u;
        L.WVin[e] = make_float2(wk[k], vk[k]);
        key[k] = f2ord(wk[k]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {  // after the padding (same addresses, program order)
        const int e = k * 64 + lane;
        if (kept[k]) {
            if (e < j0) OA[e - e_lo] = key[k];
            else OB[e - j0] = key[k];
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = k * 64 + lane;
        const bool inA = e < j0;
        const uint32_t* O = inA ? OB : OA;
        const int olen = inA ? lenB : lenA;
        const int obase = inA ? j0 : e_lo;
        // rank r: samples of the other run before (W_e, e)
        const uint32_t T = key[k] + (inA ? 0u : 1u);
        int r = 0;
#pragma unroll
        for (int step = N / 2; step >= 1; step >>= 1) r = (O[r + step - 1] < T) ? r + step : r;
        const int lo_own = inA ? e_lo : j0, hi_own = inA ? j0 - 1 : e_hi;
        const float2 pw = L.WVin[max(e - 1, lo_own)];        // own run, e - 1
        const float2 nw = L.WVin[min(e + 1, hi_own)];        // own run, e + 1
        const float2 po = L.WVin[obase + max(r - 1, 0)];     // other run, rank r - 1
        const float2 no = L.WVin[obase + min(r, olen - 1)];  // other run, rank r
        const bool hpw = e > lo_own, hnw = e < hi_own, hpo = r > 0, hno = r < olen;
        // the later predecessor and the earlier successor in (W, e) order
        const bool po_later = (po.x > pw.x) || (inA && po.x == pw.x);
        const bool nw_first = (nw.x < no.x) || (inA && nw.x == no.x);
        const float2 P = (hpo && (!hpw || po_later)) ? po : pw;
        const float2 S = (hnw && (!hno || nw_first)) ? nw : no;
        const float w = wk[k], v = vk[k];
        const bool hit = ((hpw || hpo) & (fabsf(__fsub_rn(w, P.x)) < th.zeta) & (__fsub_rn(P.y, v) > th.beta)) |
                         ((hnw || hno) & (fabsf(__fsub_rn(w, S.x)) < th.zeta) & (__fsub_rn(S.y, v) > th.beta));
        if (kept[k] & hit) stg1(Mv + pofs[k]);
    }
    wave_lds_sync();
}

template <int K>
__device__ __forceinline__ void scanline_plain(const float* __restrict__ D, int H, int W,
                                               uint8_t* __restrict__ Mv, int cx, int cy, float c, float s,
                                               float r, int h, int n, const Thresholds& th, const WaveLds& L,
                                               int lane) {
    constexpr int N = 64 * K;
    const float NaN = __int_as_float(0x7fc00000);
    float wk[K], vk[K];
    uint64_t vmask[K];
    bool kept[K];
    uint32_t pofs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = k * 64 + lane;
        const float gf = (float)(e - h);
        const int ix = (int)rintf(__fadd_rn((float)cx, __fmul_rn(c, gf)));
        const int iy = (int)rintf(__fadd_rn((float)cy, __fmul_rn(s, gf)));
        const bool valid = (e < n) & ((uint32_t)ix < (uint32_t)W) & ((uint32_t)iy < (uint32_t)H);
        const uint32_t po = (uint32_t)iy * (uint32_t)W + (uint32_t)ix;  // H * W < 2^32
        const float Vr = ldg(D + (valid ? po : 0u));  // a dropped sample reads pixel 0 and is discarded
        pofs[k] = po;
        vk[k] = valid ? Vr : 0.0f;
        wk[k] = valid ? __fsub_rn(gf, __fmul_rn(r, Vr)) : NaN;
        vmask[k] = __ballot(valid);
        kept[k] = valid;
    }
    // descents W_e < W_{e-1} (NaN compares false) split the kept samples,
    // which form one contiguous range of offsets, into runs of
    // non-decreasing W
    uint64_t dm[K];
    float wprev[K];
    int nvalid = 0, e_lo = -1, ndesc = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float fill =
            k > 0 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wk[k > 0 ? k - 1 : 0]), 63)) : NaN;
        wprev[k] = wave_up1(wk[k], fill);
        dm[k] = __ballot(wk[k] < wprev[k]);
        ndesc += __popcll(dm[k]);
        nvalid += __popcll(vmask[k]);
        if (vmask[k] && e_lo < 0) e_lo = k * 64 + __ffsll((unsigned long long)vmask[k]) - 1;
    }
    if (nvalid == 0) return;
    const int e_hi = e_lo + nvalid - 1;
    if (ndesc == 0) {
        // one run: the offsets are already in (W, g) order
        uint32_t po[K];
#pragma unroll
        for (int k = 0; k < K; ++k) po[k] = pofs[k];
        test_sorted<K>(Mv, wk, vk, po, th);
        return;
    }
    if (ndesc == 1) {
        int j0 = 0;  // the descent: B's first offset
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (dm[k]) j0 = k * 64 + __ffsll((unsigned long long)dm[k]) - 1;
        two_runs<K>(Mv, wk, vk, kept, pofs, e_lo, j0, e_hi, th, L, lane);
        return;
    }
    // three or more runs: through LDS
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = k * 64 + lane;
        L.WVin[e] = make_float2(wk[k], vk[k]);
        L.Oin[e] = f2ord(wk[k]);
    }
    wave_lds_sync();
    order_test_lds<K, 0>(Mv, W, cx, cy, c, s, h, th, L, lane, wk, vk, vmask, kept, pofs);
}

template <int KMAX>
constexpr int waves_per_block() { return KMAX >= 16 ? 2 : 4; }

// The short-scanline forms (LDS allows 8 blocks of 4 wavefronts per CU) are
// held to the hardware's 8 wavefronts per SIMD: the compiler then keeps to 96
// scalar registers, spilling a few more into VGPR lanes.  The pass is bound
// by chains of dependent loads (gather, LDS exchanges, merge searches), so
// the extra wavefronts pay: c1 scanline pass 31.0 -> 26.6 us.  The K = 4 and
// K = 8 forms are held to the 6 and 4 wavefronts per SIMD they reached before
// their three-quarter forms (K = 3, 6) were added, which would otherwise cost
// each a wavefront (80 -> 90 and 128 -> 136 VGPRs; the K = 8 form now spills
// 8 bytes per lane to scratch): 3840x2160 x15 scanline pass 1.91 -> 1.88 ms.
template <int KMAX>
constexpr int min_waves_per_simd() { return KMAX <= 2 ? 8 : KMAX == 4 ? 6 : KMAX == 8 ? 4 : 1; }

// (W, V) pair arrays per wavefront in LDS: the inputs WVin and the sorted
// WVs.  The long-scanline forms are limited by LDS, so their sorted array
// shares the input array's storage (every path reads what it needs of the
// inputs before writing the sorted values); c2 (K = 8) then fits 4 blocks per
// CU instead of 3.
template <int KMAX>
constexpr int lds_arrays() { return KMAX >= 4 ? 1 : 2; }

constexpr int kGroup = 4;  // consecutive work items per wavefront visit

// The batched kernel's prologue (a prefix over up to 1024 frames) is paid per
// block, so its short-scanline forms run 8 wavefronts per block (measured on
// 64 mixed frames: 3.06 -> 2.68 ms); for K = 8 that would leave one block per
// CU (LDS), so those keep the single-frame shape.
template <int KMAX>
constexpr int batched_waves_per_block() { return KMAX <= 4 ? 8 : waves_per_block<KMAX>(); }

// The scanline of candidate `pix` of view v of frame f.
// run_check (thinning only): false when the caller has found the candidate
// to be a head with no candidate at g = +1, whose window is the plain one.
template <int KMAX, int G>
__device__ __forceinline__ void scan_item(const FrameDesc& f, int v, uint32_t pix,
                                          const ViewTable& vt, const Thresholds& th,
                                          const WaveLds& L, int lane, bool run_check = true) {
    const int W = f.W, H = f.H;
    const int cy = (int)(pix >> 16);  // list entries are packed (y << 16) | x
    const int cx = (int)(pix & 0xffffu);
    const int h = f.h[v];
    uint8_t* Mv = f.M + (size_t)v * H * W;
    int n = 2 * h + 1;
    if (G && th.thin && run_check) {
        n = thin_window(f.D, H, W, cx, cy, vt.c[v], vt.s[v], h, th.q_min, lane);
        if (n == 0) return;  // uniform: a follower is not scanned
    }
    // the register class holds the view's longest window; a shorter one
    // (most merged windows) takes the smaller K
    if constexpr (KMAX == 2 && G == 0) {
        if (n <= 64)
            scanline_plain<1>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
        else
            scanline_plain<2>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
    } else if constexpr (KMAX == 2) {
        if (n <= 64)
            scanline<1, G>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
        else
            scanline<2, G>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
    } else if constexpr ((KMAX == 4 || KMAX == 8) && G == 0) {
        // three quarters of the class's slots when they hold the scanline
        // (the class's registers are sized for KMAX either way)
        constexpr int K3 = KMAX * 3 / 4;
        if (n <= 64 * K3)
            scanline<K3, 0>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
        else
            scanline<KMAX, 0>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
    } else {
        scanline<KMAX, G>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
    }
}

// Segment `lo` (class-local, class-major order) of class cls: its view and
// its physical segment index.
__device__ __forceinline__ void segment_of(const FrameDesc& f, int cls, int lo, int* v, int* seg) {
    const int C = f.ll.copies;
    // lo / C (lo < kMaxSegments); ceil(2^32 / C) does not fit 32 bits for C = 1
    const int q = C == 1 ? lo : (int)__umulhi((uint32_t)lo, f.copies_magic);
    *v = f.vord[f.cls_start[cls] + q];
    *seg = *v * C + (lo - q * C);
}

// One frame, the views of scan class cls: a flat walk over every
// (view, candidate) pair of the class.
template <int KMAX, int G>
__global__ __launch_bounds__(64 * waves_per_block<KMAX>(), min_waves_per_simd<KMAX>()) void k_scanlines(
    FrameDesc f, int n_views, ViewTable vt, Thresholds th, int cls) {
    constexpr int WPB = waves_per_block<KMAX>();
    constexpr int NT = 64 * WPB;
    __shared__ float2 lds[WPB][lds_arrays<KMAX>()][64 * KMAX];
    __shared__ uint32_t okeys[WPB][64 * KMAX];
    __shared__ int runs[WPB][kMaxRunsCap + 1];
    __shared__ int pre[kMaxSegments + 1];
    __shared__ int segvs[kMaxSegments];  // class segment j: (view << 16) | physical segment
    const int C = f.ll.copies;
    const int seg0 = f.cls_start[cls] * C;
    const int nseg = (f.cls_start[cls + 1] - f.cls_start[cls]) * C;
    const int base = f.prefix[seg0];
    for (int j = threadIdx.x; j <= nseg; j += NT) {
        pre[j] = f.prefix[seg0 + j] - base;
        if (j < nseg) {
            const int v = f.vord[f.cls_start[cls] + j / C];
            segvs[j] = (v << 16) | (v * C + j % C);
        }
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    constexpr int NA = lds_arrays<KMAX>();
    const WaveLds L{lds[wave][0], okeys[wave], lds[wave][NA - 1], runs[wave]};
    // one item: the class-list index t, its segment found by stepping forward from lo
    auto item = [&](int t, int& lo, bool run_check) {
        while (lo + 1 < nseg && pre[lo + 1] <= t) ++lo;
        const int sv = segvs[lo];
        const int v = sv >> 16, seg = sv & 0xffff;
        const uint32_t pix = f.lists[(size_t)seg * f.ll.cap + (size_t)(t - pre[lo])];
        scan_item<KMAX, G>(f, v, pix, vt, th, L, lane, run_check);
    };
    // Thinning: one load round tests the pixels at g = -1 (lane 2i) and
    // g = +1 (lane 2i + 1) of item g0 + i of a group.  Bit 2i of the result:
    // the item is a follower; bit 2i + 1: it has a candidate at g = +1.
    auto thin_group = [&](int g0, int g1, int lo) {
        bool is_c = false;
        if (lane < 2 * (g1 - g0)) {
            const int t = g0 + (lane >> 1);
            int l = lo;
            while (l + 1 < nseg && pre[l + 1] <= t) ++l;
            const int sv = segvs[l];
            const int v = sv >> 16, seg = sv & 0xffff;
            const uint32_t pix = f.lists[(size_t)seg * f.ll.cap + (size_t)(t - pre[l])];
            is_c = candidate_at(f.D, f.H, f.W, (int)(pix & 0xffffu), (int)(pix >> 16), vt.c[v], vt.s[v],
                                (lane & 1) ? 1 : -1, th.q_min);
        }
        return (uint32_t)__ballot(is_c);
    };
    auto seg_of = [&](int t) {  // last segment with pre <= t
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= t) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    // Workgroups are dealt to the 8 dies (XCDs, each with its own L2) in
    // turn.  For a frame whose D exceeds what the dies' L2s hold together,
    // die x = blockIdx % 8 takes the x-th eighth of every view's items; a
    // view's items are ordered by row band, so a die works on about one eighth
    // of the frame's rows of every view (its own part of D in its L2) with the
    // same mix of scanline lengths as the others (3840x2160 x 15: 2.67 ->
    // 2.44 ms).  For smaller frames the split costs more than it saves (c1
    // 34.4 -> 36.8 us), and all wavefronts share one list.
    constexpr int kDies = 8;
    constexpr size_t kDieSplitBytes = size_t(16) << 20;
    const bool split = gridDim.x >= kDies && (size_t)f.H * f.W * sizeof(float) >= kDieSplitBytes;
    if (!split) {
        // Blocked round-robin: wavefront gw takes groups of kGroup consecutive
        // items at gw*kGroup, gw*kGroup + nw*kGroup, ...  All wavefronts sweep
        // the list together (a small live working set of D), and within a
        // group the segment is found by stepping forward.
        const int total = pre[nseg];
        const int nw = gridDim.x * WPB;
        const int gw = blockIdx.x * WPB + wave;
        for (int g0 = gw * kGroup; g0 < total; g0 += nw * kGroup) {
            const int g1 = min(total, g0 + kGroup);
            int lo = seg_of(g0);
            if (G && th.thin) {
                const uint32_t tb = thin_group(g0, g1, lo);
                for (int t = g0; t < g1; ++t) {
                    const uint32_t b = tb >> (2 * (t - g0));
                    if (!(b & 1u)) item(t, lo, (b & 2u) != 0);  // followers are skipped
                }
            } else {
                for (int t = g0; t < g1; ++t) item(t, lo, true);
            }
        }
        return;
    }
    // dst: die-local prefix over the class's views; gst: class-list index of
    // the die's first item of each view
    __shared__ int dst[OCCL_MAX_VIEWS + 1];
    __shared__ int gst[OCCL_MAX_VIEWS];
    const int nvc = f.cls_start[cls + 1] - f.cls_start[cls];
    const int die = (int)(blockIdx.x % kDies);
    if (threadIdx.x < 64) {  // one wavefront: nvc <= 64
        const int j = threadIdx.x;
        int a = 0, cnt = 0;
        if (j < nvc) {
            const int vs = pre[j * C], ve = pre[(j + 1) * C];
            a = vs + (int)((long long)(ve - vs) * die / kDies);
            cnt = vs + (int)((long long)(ve - vs) * (die + 1) / kDies) - a;
        }
        int x = cnt;  // inclusive scan over the views
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (j >= d) x += y;
        }
        if (j < nvc) {
            dst[j] = x - cnt;
            gst[j] = a;
        }
        if (j == nvc - 1) dst[nvc] = x;
        if (nvc == 0 && j == 0) dst[0] = 0;
    }
    __syncthreads();
    const int total = dst[nvc];
    // blocked round-robin within the die; view and segment found by stepping forward
    const int nw = (int)((gridDim.x - die + kDies - 1) / kDies) * WPB;
    const int gw = (int)(blockIdx.x / kDies) * WPB + wave;
    for (int g0 = gw * kGroup; g0 < total; g0 += nw * kGroup) {
        const int g1 = min(total, g0 + kGroup);
        int j = 0;  // view of the group's first item (last with dst <= g0)
        while (j + 1 < nvc && dst[j + 1] <= g0) ++j;
        int lo = seg_of(gst[j] + (g0 - dst[j]));
        for (int tl = g0; tl < g1; ++tl) {
            while (j + 1 < nvc && dst[j + 1] <= tl) ++j;
            item(gst[j] + (tl - dst[j]), lo, true);
        }
    }
}

// Every frame of a batch, the views of scan class cls: the flat work list
// is frame-major; frame sizes come from each frame's prefix, segments are
// located in the frame's prefix in global memory.
template <int KMAX, int G>
__global__ __launch_bounds__(64 * batched_waves_per_block<KMAX>(), min_waves_per_simd<KMAX>()) void k_scanlines_batched(
    const FrameDesc* __restrict__ table, int n_frames, int n_views, ViewTable vt, Thresholds th,
    int cls) {
    constexpr int WPB = batched_waves_per_block<KMAX>();
    constexpr int NT = 64 * WPB;
    __shared__ float2 lds[WPB][lds_arrays<KMAX>()][64 * KMAX];
    __shared__ uint32_t okeys[WPB][64 * KMAX];
    __shared__ int runs[WPB][kMaxRunsCap + 1];
    __shared__ int fpre[kMaxBatch + 1];
    __shared__ int wsum[WPB];
    {  // exclusive prefix of the per-frame item counts of this class
        constexpr int PER = (kMaxBatch + NT - 1) / NT;
        const int t = threadIdx.x, ln = t & 63, wv = t >> 6;
        int cnt[PER];
        int sum = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int fi = t * PER + j;
            int cc = 0;
            if (fi < n_frames) {
                const FrameDesc& f = table[fi];
                const int C = f.ll.copies;
                const int s0 = f.cls_start[cls] * C, s1 = f.cls_start[cls + 1] * C;
                cc = f.prefix[s1] - f.prefix[s0];
            }
            cnt[j] = cc;
            sum += cc;
        }
        int x = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (ln >= d) x += y;
        }
        if (ln == 63) wsum[wv] = x;
        __syncthreads();
        int run = x - sum;
        for (int w = 0; w < wv; ++w) run += wsum[w];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int fi = t * PER + j;
            if (fi < n_frames) fpre[fi] = run;
            run += cnt[j];
        }
        if (t == NT - 1) fpre[n_frames] = run;
    }
    __syncthreads();
    const int total = fpre[n_frames];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    constexpr int NA = lds_arrays<KMAX>();
    const WaveLds L{lds[wave][0], okeys[wave], lds[wave][NA - 1], runs[wave]};
    // Workgroups are dealt to the 8 dies (XCDs, each with its own L2) in
    // turn, so die x = blockIdx % 8 takes the x-th eighth of the frame-major
    // list: each L2 then holds only its own frames' D.  Within a die, blocked
    // round-robin (see k_scanlines).  Every item is in exactly one eighth;
    // with fewer than 8 blocks the whole list is dealt to all of them.
    constexpr int kDies = 8;
    const bool split = gridDim.x >= kDies;
    const int die = split ? (int)(blockIdx.x % kDies) : 0;
    const int nb = split ? (int)((gridDim.x - die + kDies - 1) / kDies) : (int)gridDim.x;
    const int bi = split ? (int)(blockIdx.x / kDies) : (int)blockIdx.x;
    const int c0 = split ? (int)((long long)total * die / kDies) : 0;
    const int c1 = split ? (int)((long long)total * (die + 1) / kDies) : total;
    const int nw = nb * WPB;
    const int gw = bi * WPB + wave;
    int fi = 0;
    for (int g0 = c0 + gw * kGroup; g0 < c1; g0 += nw * kGroup) {
        const int g1 = min(c1, g0 + kGroup);
        int fi_cur = -1, lo = 0, nseg = 0, seg0 = 0, pbase = 0;
        for (int t = g0; t < g1; ++t) {
            if (fi_cur < 0 || t >= fpre[fi_cur + 1]) {
                // frame of item t (last with fpre <= t), then its segment by binary search
                int a = fi, b = n_frames - 1;
                while (a < b) {
                    const int mid = (a + b + 1) >> 1;
                    if (fpre[mid] <= t) a = mid; else b = mid - 1;
                }
                fi = fi_cur = a;
                const FrameDesc& f = table[fi_cur];
                const int C = f.ll.copies;
                seg0 = f.cls_start[cls] * C;
                nseg = (f.cls_start[cls + 1] - f.cls_start[cls]) * C;
                pbase = f.prefix[seg0];
                const int u = t - fpre[fi_cur];
                int p = 0, q = nseg - 1;
                while (p < q) {
                    const int mid = (p + q + 1) >> 1;
                    if (f.prefix[seg0 + mid] - pbase <= u) p = mid; else q = mid - 1;
                }
                lo = p;
            }
            const FrameDesc& f = table[fi_cur];
            const int u = t - fpre[fi_cur];
            while (lo + 1 < nseg && f.prefix[seg0 + lo + 1] - pbase <= u) ++lo;
            int v, seg;
            segment_of(f, cls, lo, &v, &seg);
            const uint32_t pix =
                f.lists[(size_t)seg * f.ll.cap + (size_t)(u - (f.prefix[seg0 + lo] - pbase))];
            scan_item<KMAX, G>(f, v, pix, vt, th, L, lane);
        }
    }
}

// ---------------------------------------------------------------------------
// Fused pass: Eqs. (1)-(6) of every view of one tile of kFusedRows x 256
// pixels in one block, for frames whose views all have scanlines of at most
// 128 samples (plain form).  Per tile:
//   1. the block loads the tile (one wavefront per row, as the edge pass),
//      applies Eq. (1) and the magnitude half of Eq. (2), and compacts the
//      strong pixels (with their differences) into LDS;
//   2. one lane per strong pixel applies the direction half of Eq. (2) for
//      every view and appends the candidates to an LDS queue, so the
//      per-view work scales with the strong pixels, not with the tile;
//   3. the wavefronts take queue entries as they finish their previous one
//      and run those scanlines, gathering D from global memory.
// A tile with more strong pixels than the queue holds for all views runs 2
// and 3 in rounds over slices of its strong pixels.  No candidate list,
// list counter, prefix or second launch is involved.  Hits are byte stores
// of 1 into masks that a fill kernel has cleared before the pass (a
// scanline can write up to h pixels outside its tile, so the tile cannot
// clear its own pixels).
// Tiles are handed out by tickets: the flat tile list of the launch is cut
// into kFusedParts contiguous parts, block b starts on part b % kFusedParts
// (blocks are dealt to the 8 dies in turn, so each die mostly works on one
// part and keeps that part's D in its L2) and moves on to the other parts
// when its own is exhausted.
// ---------------------------------------------------------------------------
constexpr int kFusedParts = 8;

template <int ROWS>
struct FusedShared {
    static constexpr int kQueue = ROWS * kEdgeCols;  // candidate entries per round (the tile's pixels)
    uint32_t queue[kQueue];       // (v << 12) | (row << 8) | column of the tile
    uint16_t spix[kQueue];        // strong pixels: (row << 8) | column
    int ns;                       // strong pixels of the tile
    int qn;                       // entries in the queue
    int take;                     // entries handed to wavefronts
    int tile, fi;                 // the block's current tile (-1: done) and its frame
    int next, next_fi;            // the next ones (fetched while the current one runs)
};

// Next tile for block `part0`'s thread 0: tickets of part p run from
// pbeg[p] to pbeg[p + 1]; exhausted parts are skipped in turn.
__device__ __forceinline__ int fused_ticket(unsigned* tickets, const int* pbeg, int& part, int part0) {
    for (int k = 0; k < kFusedParts; ++k) {
        const int p = (part0 + ((part - part0 + kFusedParts) % kFusedParts)) % kFusedParts;
        const int t = pbeg[p] + (int)atomicAdd(&tickets[p * 32], 1u);
        if (t < pbeg[p + 1]) return t;
        part = (part + 1) % kFusedParts;
        if (part == part0) break;
    }
    return -1;
}

// Frame of flat tile t: the last frame whose first tile is at most t.
__device__ __forceinline__ int fused_frame_of(const int* begin, int n_frames, int t) {
    int a = 0, b = n_frames - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (begin[mid] <= t) a = mid; else b = mid - 1;
    }
    return a;
}

// One tile (bx, by) of frame f.  Every thread of the block calls it.
// exy: kQueue entries of LDS free until the first scanline of the tile (the
// scanline scratch), holding the strong pixels' differences meanwhile.
// On entry S.qn and S.take are 0 and S.ns holds no other tile's pixels; on
// return S.ns is 0 again and S.qn, S.take are cleared by the caller after
// the block's next barrier.
template <int ROWS>
__device__ __forceinline__ void fused_tile(const FrameDesc& f, int bx, int by, int n_views, const ViewTable& vt,
                                           const Thresholds& th, const WaveLds& L, FusedShared<ROWS>& S,
                                           float2* exy, int wave, int lane) {
    constexpr int kQ = FusedShared<ROWS>::kQueue;
    const int H = f.H, W = f.W;
    const int y = by * ROWS + wave;
    const int x0 = bx * kEdgeCols + lane * 4;
    const bool live = (y < H) && (x0 < W);
    const EdgeIn in = edge_load(f, bx, by);
    // Eq. (1) and the magnitude half of Eq. (2) (q >= q_min is sqrt_rn(q) > gamma)
    float ex[4], ey[4];
    unsigned strong = 0;
    {
        const bool next_row = (y + 1 < H);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float right = (j < 3) ? in.d0[j + 1] : in.dn;
            ex[j] = (x0 + j + 1 < W) ? __fsub_rn(right, in.d0[j]) : 0.0f;
            ey[j] = next_row ? __fsub_rn(in.d1[j], in.d0[j]) : 0.0f;
            const float q = __fadd_rn(__fmul_rn(ex[j], ex[j]), __fmul_rn(ey[j], ey[j]));
            strong |= (live && (x0 + j < W) && (q >= th.q_min)) ? (1u << j) : 0u;
        }
    }
    // 1. the strong pixels and their differences
    {
        uint64_t b[4];
        int tot = 0, off = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b[j] = __ballot((strong >> j) & 1u);
            tot += __popcll(b[j]);
            off += (int)lanes_below(b[j]);
        }
        if (tot) {  // uniform
            int base = 0;
            if (lane == 0) base = atomicAdd(&S.ns, tot);
            int i = __builtin_amdgcn_readfirstlane(base) + off;
            const uint32_t p0 = ((uint32_t)wave << 8) | (uint32_t)(lane * 4);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if ((strong >> j) & 1u) {
                    S.spix[i] = (uint16_t)(p0 + (uint32_t)j);
                    exy[i] = make_float2(ex[j], ey[j]);
                    ++i;
                }
            }
        }
    }
    __syncthreads();
    const int ns = S.ns;
    const int per = kQ / n_views;  // strong pixels per round: their candidates fit the queue
    for (int pa = 0; pa < ns; pa += per) {
        const int pb = min(ns, pa + per);
        // 2. the direction half of Eq. (2), one lane per strong pixel
        for (int i0 = pa + wave * 64; i0 < pb; i0 += ROWS * 64) {
            const int i = i0 + lane;
            const bool ok = i < pb;
            const uint32_t p = S.spix[ok ? i : pa];
            float gx, gy;
            if (pa == 0) {
                const float2 g = exy[ok ? i : 0];
                gx = g.x;
                gy = g.y;
            } else {  // the scanlines of the first round used exy: from D again
                const int py = by * ROWS + (int)(p >> 8), px = bx * kEdgeCols + (int)(p & 255u);
                const float* d = f.D + (size_t)py * W + px;
                const float d0 = ldg(d);
                gx = (px + 1 < W) ? __fsub_rn(ldg(d + 1), d0) : 0.0f;
                gy = (py + 1 < H) ? __fsub_rn(ldg(d + W), d0) : 0.0f;
            }
            for (int v = 0; v < n_views; ++v) {
                const float dot = __fadd_rn(__fmul_rn(gx, vt.c[v]), __fmul_rn(gy, vt.s[v]));
                const bool c = ok && (dot > 0.0f);
                const uint64_t bm = __ballot(c);
                if (bm == 0) continue;  // uniform
                int base = 0;
                if (lane == 0) base = atomicAdd(&S.qn, __popcll(bm));
                base = __builtin_amdgcn_readfirstlane(base);
                if (c) S.queue[base + (int)lanes_below(bm)] = ((uint32_t)v << 12) | p;
            }
        }
        __syncthreads();
        // 3. wavefronts take entries as they finish their previous one
        const int nq = S.qn;
        for (;;) {
            int i = 0;
            if (lane == 0) i = atomicAdd(&S.take, 1);
            i = __builtin_amdgcn_readfirstlane(i);
            if (i >= nq) break;
            const uint32_t ent = S.queue[i];
            const int v = (int)(ent >> 12);
            const int cy = by * ROWS + (int)((ent >> 8) & 15u);
            const int cx = bx * kEdgeCols + (int)(ent & 255u);
            const int h = f.h[v];
            const int n = 2 * h + 1;
            uint8_t* Mv = f.M + (size_t)v * H * W;
            if (n <= 64)
                scanline_plain<1>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
            else
                scanline_plain<2>(f.D, H, W, Mv, cx, cy, vt.c[v], vt.s[v], vt.r[v], h, n, th, L, lane);
        }
        if (pa + per < ns) {  // another round: the queue is reused
            __syncthreads();
            if (threadIdx.x == 0) {
                S.qn = 0;
                S.take = 0;
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) S.ns = 0;  // every thread read ns before the barrier after step 2
}

// All frames of the launch (one for a single frame): a persistent grid
// walks the tiles by tickets.  tickets: kFusedParts counters 128 bytes
// apart, zero at launch (the mask fill kernel clears them).
template <int ROWS>
__global__ __launch_bounds__(64 * ROWS, 8) void k_fused(const FrameDesc* __restrict__ table, int n_frames,
                                                        int total_tiles, int n_views, ViewTable vt, Thresholds th,
                                                        unsigned* tickets) {
    __shared__ FusedShared<ROWS> S;
    __shared__ int begin[kMaxBatch + 1];
    __shared__ int pbeg[kFusedParts + 1];
    __shared__ float2 lds[ROWS][2][128];
    __shared__ uint32_t okeys[ROWS][128];
    __shared__ int runs[ROWS][kMaxRunsCap + 1];
    static_assert(sizeof(lds) / sizeof(float2) == FusedShared<ROWS>::kQueue, "exy spans the scanline scratch");
    for (int i = threadIdx.x; i < n_frames; i += blockDim.x) begin[i] = table[i].block_begin;
    if (threadIdx.x == 0) begin[n_frames] = total_tiles;
    if (threadIdx.x <= kFusedParts) pbeg[threadIdx.x] = (int)((long long)total_tiles * threadIdx.x / kFusedParts);
    const int part0 = (int)(blockIdx.x % kFusedParts);
    int part = part0;  // thread 0's current part
    __syncthreads();
    if (threadIdx.x == 0) {
        S.ns = 0;
        S.qn = 0;
        S.take = 0;
        S.tile = fused_ticket(tickets, pbeg, part, part0);
        S.fi = S.tile < 0 ? 0 : fused_frame_of(begin, n_frames, S.tile);
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const WaveLds L{lds[wave][0], okeys[wave], lds[wave][1], runs[wave]};
    for (;;) {
        const int t = S.tile;
        if (t < 0) break;
        const int fi = S.fi;
        if (threadIdx.x == 0) {
            // the previous tile's queue counters (every wavefront has passed
            // the barrier that ended that tile) and the next ticket
            S.qn = 0;
            S.take = 0;
            S.next = fused_ticket(tickets, pbeg, part, part0);
            S.next_fi = S.next < 0 ? 0 : fused_frame_of(begin, n_frames, S.next);
        }
        const FrameDesc& f = table[fi];
        const int local = t - begin[fi];
        fused_tile<ROWS>(f, local % f.gx, local / f.gx, n_views, vt, th, L, S, &lds[0][0][0], wave, lane);
        // every thread read S.tile and S.fi before the tile's first barrier
        if (threadIdx.x == 0) {
            S.tile = S.next;
            S.fi = S.next_fi;
        }
        __syncthreads();
    }
}

// Clears the masks of the launch's frames (16-byte stores where aligned):
// block (x, fi) clears bytes [x * kClearChunkBytes, (x + 1) * kClearChunkBytes) of
// frame fi's masks; block (0, 0) also clears the fused pass's tickets.
__global__ __launch_bounds__(256) void k_clear_masks(const FrameDesc* __restrict__ table, int n_views,
                                                     unsigned* tickets) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < kFusedParts) tickets[threadIdx.x * 32] = 0u;
    const FrameDesc& f = table[blockIdx.y];
    const long long bytes = (long long)f.H * f.W * n_views;
    const long long o0 = (long long)blockIdx.x * kClearChunkBytes;
    if (o0 >= bytes) return;
    const long long o1 = o0 + kClearChunkBytes < bytes ? o0 + kClearChunkBytes : bytes;
    uint8_t* M = f.M;
    if ((((uintptr_t)M) & 15) == 0) {
        long long o = o0 + (long long)threadIdx.x * 16;
        for (; o + 16 <= o1; o += 256 * 16) *reinterpret_cast<uint4*>(M + o) = make_uint4(0u, 0u, 0u, 0u);
        for (; o < o1; ++o) M[o] = 0;  // the frame's last partial vector: one thread
    } else {
        for (long long o = o0 + threadIdx.x; o < o1; o += 256) M[o] = 0;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
ListLayout make_list_layout(int H, int W, int n_views, int edge_rows) {
    ListLayout ll;
    ll.edge_rows = edge_rows;
    const int block_rows = (H + edge_rows - 1) / edge_rows;
    // Bands of block rows: enough that one list counter takes the atomics of
    // about kWavesPerBand edge-pass wavefronts, no more (every extra segment
    // costs the frame's prefix and the scanline pass's segment tables).
    const long long waves = (long long)block_rows * edge_rows * ((W + kEdgeCols - 1) / kEdgeCols);
    const long long want = (waves + kWavesPerBand - 1) / kWavesPerBand;
    int copies = want < kMaxCopies ? (int)want : kMaxCopies;
    if (copies > kMaxSegments / (n_views > 0 ? n_views : 1)) copies = kMaxSegments / (n_views > 0 ? n_views : 1);
    if (copies > block_rows) copies = block_rows;
    if (copies < 1) copies = 1;
    ll.block_rows_per_copy = (block_rows + copies - 1) / copies;
    ll.copies = (block_rows + ll.block_rows_per_copy - 1) / ll.block_rows_per_copy;
    ll.cap = (size_t)ll.block_rows_per_copy * edge_rows * (size_t)W;
    return ll;
}

void describe_frame(FrameDesc* f, const float* D, uint8_t* M, int H, int W, int n_views,
                    const int* Ls, int edge_rows, int thin) {
    f->D = D;
    f->M = M;
    f->H = H;
    f->W = W;
    f->ll = make_list_layout(H, W, n_views, edge_rows);
    f->copies_magic = f->ll.copies > 1
                          ? (uint32_t)(((1ull << 32) + (uint64_t)f->ll.copies - 1) / (uint64_t)f->ll.copies)
                          : 0u;  // unused for one copy
    f->gx = (W + kEdgeCols - 1) / kEdgeCols;
    f->gy = (H + edge_rows - 1) / edge_rows;
    f->block_begin = 0;
    for (int v = 0; v < OCCL_MAX_VIEWS; ++v) {
        f->h[v] = v < n_views ? Ls[v] / 2 : 0;
        f->vord[v] = 0;
    }
    int k = 0;
    for (int ci = 0; ci < kNumClasses; ++ci) {
        f->cls_start[ci] = k;
        for (int v = 0; v < n_views; ++v)
            if (scan_class(f->h[v], thin) == ci) f->vord[k++] = v;
    }
    f->cls_start[kNumClasses] = k;
}

hipError_t launch_edges(hipStream_t st, const FrameDesc& f, int n_views, const ViewTable& vt,
                        float q_min) {
    hipLaunchKernelGGL(k_edges, dim3(f.gx, f.gy), dim3(64 * f.ll.edge_rows), 0, st, f, n_views, vt, q_min);
    return hipGetLastError();
}

int edges_batched_blocks_per_cu(int edge_rows) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_edges_batched, 64 * edge_rows, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

hipError_t launch_edges_batched(hipStream_t st, const FrameDesc* table, int n_frames,
                                int total_blocks, int n_views, const ViewTable& vt, float q_min,
                                int edge_rows, int n_blocks) {
    hipLaunchKernelGGL(k_edges_batched, dim3(n_blocks), dim3(64 * edge_rows), 0, st, table,
                       n_frames, total_blocks, n_views, vt, q_min);
    hipLaunchKernelGGL(k_finish_frames, dim3(n_frames), dim3(256), 0, st, table, n_views);
    return hipGetLastError();
}

namespace {

template <int G>
hipError_t launch_scanlines_g(hipStream_t st, const FrameDesc& f, int n_views, const ViewTable& vt,
                              const Thresholds& th, int cls, int n_blocks) {
    const dim3 grid(n_blocks);
    switch (cls) {
        case 0:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines<2, G>), grid, dim3(64 * waves_per_block<2>()), 0,
                               st, f, n_views, vt, th, cls);
            break;
        case 1:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines<4, G>), grid, dim3(64 * waves_per_block<4>()), 0,
                               st, f, n_views, vt, th, cls);
            break;
        case 2:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines<8, G>), grid, dim3(64 * waves_per_block<8>()), 0,
                               st, f, n_views, vt, th, cls);
            break;
        case 3:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines<16, G>), grid, dim3(64 * waves_per_block<16>()), 0,
                               st, f, n_views, vt, th, cls);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int G>
hipError_t launch_scanlines_batched_g(hipStream_t st, const FrameDesc* table, int n_frames, int n_views,
                                      const ViewTable& vt, const Thresholds& th, int cls, int n_blocks) {
    const dim3 grid(n_blocks);
    switch (cls) {
        case 0:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines_batched<2, G>), grid,
                               dim3(64 * batched_waves_per_block<2>()), 0, st, table, n_frames, n_views, vt,
                               th, cls);
            break;
        case 1:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines_batched<4, G>), grid,
                               dim3(64 * batched_waves_per_block<4>()), 0, st, table, n_frames, n_views, vt,
                               th, cls);
            break;
        case 2:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines_batched<8, G>), grid,
                               dim3(64 * batched_waves_per_block<8>()), 0, st, table, n_frames, n_views, vt,
                               th, cls);
            break;
        case 3:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_scanlines_batched<16, G>), grid,
                               dim3(64 * batched_waves_per_block<16>()), 0, st, table, n_frames, n_views, vt,
                               th, cls);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_scanlines(hipStream_t st, const FrameDesc& f, int n_views, const ViewTable& vt,
                            const Thresholds& th, int cls, int n_blocks) {
    return (th.bilinear || th.thin || th.ns != 1)
               ? launch_scanlines_g<1>(st, f, n_views, vt, th, cls, n_blocks)
               : launch_scanlines_g<0>(st, f, n_views, vt, th, cls, n_blocks);
}

// Batched frames are never thinned.
int fused_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused<kFusedTileRows>, 64 * kFusedTileRows, 0) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

hipError_t launch_fused_stage(hipStream_t st, const FrameDesc* table, int n_frames, int total_tiles, int n_views,
                              const ViewTable& vt, const Thresholds& th, unsigned* tickets, int n_blocks,
                              int clear_blocks, int stage) {
    if (stage == 0)
        hipLaunchKernelGGL(k_clear_masks, dim3(clear_blocks, n_frames), dim3(256), 0, st, table, n_views, tickets);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fused<kFusedTileRows>), dim3(n_blocks), dim3(64 * kFusedTileRows), 0,
                           st, table, n_frames, total_tiles, n_views, vt, th, tickets);
    return hipGetLastError();
}

hipError_t launch_fused(hipStream_t st, const FrameDesc* table, int n_frames, int total_tiles, int n_views,
                        const ViewTable& vt, const Thresholds& th, unsigned* tickets, int n_blocks,
                        int clear_blocks) {
    hipError_t e = launch_fused_stage(st, table, n_frames, total_tiles, n_views, vt, th, tickets, n_blocks,
                                      clear_blocks, 0);
    if (e == hipSuccess)
        e = launch_fused_stage(st, table, n_frames, total_tiles, n_views, vt, th, tickets, n_blocks, clear_blocks, 1);
    return e;
}

hipError_t launch_scanlines_batched(hipStream_t st, const FrameDesc* table, int n_frames,
                                    int n_views, const ViewTable& vt, const Thresholds& th,
                                    int cls, int n_blocks) {
    return (th.bilinear || th.ns != 1)
               ? launch_scanlines_batched_g<1>(st, table, n_frames, n_views, vt, th, cls, n_blocks)
               : launch_scanlines_batched_g<0>(st, table, n_frames, n_views, vt, th, cls, n_blocks);
}

}  // namespace occl
