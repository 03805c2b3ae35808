// k_util.hip -- small helper kernels: statistics of D (automatic scan length,
// input validation), the edge magnitude / angle maps of Eq. (1) as outputs,
// and the confusion counts behind Eq. (7).
#include <cmath>

#include "occl_internal.h"

namespace occl {
namespace {

__device__ __forceinline__ uint32_t ford(float w) {
    const uint32_t u = __float_as_uint(w);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Statistics of D in two launches without atomics: per-block partials
// (min, max as orderable uints, non-finite count), then one block folds them.
__device__ __forceinline__ void fold_stats(uint32_t& mn, uint32_t& mx, uint32_t& bad) {
    __shared__ uint32_t red[3][4];
    for (int m = 32; m > 0; m >>= 1) {
        const uint32_t a = (uint32_t)__shfl_xor((int)mn, m, 64);
        const uint32_t b = (uint32_t)__shfl_xor((int)mx, m, 64);
        const uint32_t c = (uint32_t)__shfl_xor((int)bad, m, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
        bad += c;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = mn;
        red[1][w] = mx;
        red[2][w] = bad;
    }
    __syncthreads();
    mn = red[0][0];
    mx = red[1][0];
    bad = red[2][0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
        mn = red[0][k] < mn ? red[0][k] : mn;
        mx = red[1][k] > mx ? red[1][k] : mx;
        bad += red[2][k];
    }
}

__global__ __launch_bounds__(256) void k_stats(const float* __restrict__ D, size_t n,
                                               uint32_t* __restrict__ partial) {
    uint32_t mn = 0xffffffffu, mx = 0u, bad = 0u;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float d = D[i];
        if (!isfinite(d)) {
            ++bad;
            continue;
        }
        const uint32_t o = ford(d);
        mn = o < mn ? o : mn;
        mx = o > mx ? o : mx;
    }
    fold_stats(mn, mx, bad);
    if (threadIdx.x == 0) {
        partial[(size_t)blockIdx.x * 3 + 0] = mn;
        partial[(size_t)blockIdx.x * 3 + 1] = mx;
        partial[(size_t)blockIdx.x * 3 + 2] = bad;
    }
}

__global__ __launch_bounds__(256) void k_stats_sum(const uint32_t* __restrict__ partial, int n_blocks,
                                                   uint32_t* __restrict__ out) {
    uint32_t mn = 0xffffffffu, mx = 0u, bad = 0u;
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) {
        const uint32_t a = partial[(size_t)b * 3], c = partial[(size_t)b * 3 + 1];
        mn = a < mn ? a : mn;
        mx = c > mx ? c : mx;
        bad += partial[(size_t)b * 3 + 2];
    }
    fold_stats(mn, mx, bad);
    if (threadIdx.x == 0) {
        out[0] = mn;
        out[1] = mx;
        out[2] = bad;
    }
}

// Correctly rounded fp32 square root: the hardware estimate is within one
// ulp; the neighbour whose rounding interval holds sqrt(q) is selected with
// exact double arithmetic (a midpoint has 25 significant bits, its square 50).
__device__ __forceinline__ float sqrt_cr(float q) {
    if (!(q > 0.0f) || isinf(q)) return __builtin_sqrtf(q);
    const float s = __builtin_sqrtf(q);
    const float lo = nextafterf(s, 0.0f);
    const float hi = nextafterf(s, INFINITY);
    const double qd = (double)q;
    const double mh = 0.5 * ((double)s + (double)hi);
    const double ml = 0.5 * ((double)lo + (double)s);
    if (mh * mh <= qd) return hi;
    if (ml * ml >= qd) return lo;
    return s;
}

__global__ __launch_bounds__(256) void k_edges_out(const float* __restrict__ D, int H, int W,
                                                   float* __restrict__ E, float* __restrict__ A) {
    const size_t n = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i % W);
        const float d = D[i];
        const float ex = (x + 1 < W) ? __fsub_rn(D[i + 1], d) : 0.0f;
        const float ey = (y + 1 < H) ? __fsub_rn(D[i + W], d) : 0.0f;
        if (E) E[i] = sqrt_cr(__fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey)));
        if (A) A[i] = atan2f(ey, ex);
    }
}

// Confusion counts: per-block partial TP / FP / FN (16 mask bytes per lane
// per step), then one block sums the partials in a fixed order; TN = n minus
// the other three.  No atomics, so the result is deterministic.
__device__ __forceinline__ uint32_t nz_bits(uint32_t w) {  // bit b: byte b of w is nonzero
    return (uint32_t)((w & 0xffu) != 0) | ((uint32_t)((w & 0xff00u) != 0) << 1) |
           ((uint32_t)((w & 0xff0000u) != 0) << 2) | ((uint32_t)((w & 0xff000000u) != 0) << 3);
}

__global__ __launch_bounds__(256) void k_confusion(const uint8_t* __restrict__ pred,
                                                   const uint8_t* __restrict__ ref, size_t n,
                                                   unsigned long long* __restrict__ partial) {
    __shared__ unsigned long long red[3][4];
    unsigned long long tp = 0, fp = 0, fn = 0;
    const bool vec = ((reinterpret_cast<uintptr_t>(pred) | reinterpret_cast<uintptr_t>(ref)) & 15) == 0;
    const size_t nv = vec ? n / 16 : 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (size_t)gridDim.x * blockDim.x) {
        const uint4 a = reinterpret_cast<const uint4*>(pred)[i];
        const uint4 b = reinterpret_cast<const uint4*>(ref)[i];
        const uint32_t P = nz_bits(a.x) | (nz_bits(a.y) << 4) | (nz_bits(a.z) << 8) | (nz_bits(a.w) << 12);
        const uint32_t T = nz_bits(b.x) | (nz_bits(b.y) << 4) | (nz_bits(b.z) << 8) | (nz_bits(b.w) << 12);
        tp += __popc(P & T);
        fp += __popc(P & ~T);
        fn += __popc(~P & T & 0xffffu);
    }
    for (size_t i = nv * 16 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const bool p = pred[i] != 0, t = ref[i] != 0;
        tp += (p && t);
        fp += (p && !t);
        fn += (!p && t);
    }
    for (int m = 32; m > 0; m >>= 1) {
        tp += __shfl_xor(tp, m, 64);
        fp += __shfl_xor(fp, m, 64);
        fn += __shfl_xor(fn, m, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = tp;
        red[1][w] = fp;
        red[2][w] = fn;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[threadIdx.x][k];
        partial[(size_t)blockIdx.x * 3 + threadIdx.x] = t;
    }
}

// Integer sums, so the fold order never changes the result.
__global__ __launch_bounds__(256) void k_confusion_sum(const unsigned long long* __restrict__ partial,
                                                       int n_blocks, size_t n,
                                                       unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[3][4];
    unsigned long long t[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x)
        for (int j = 0; j < 3; ++j) t[j] += partial[(size_t)b * 3 + j];
    for (int m = 32; m > 0; m >>= 1)
        for (int j = 0; j < 3; ++j) t[j] += __shfl_xor(t[j], m, 64);
    if ((threadIdx.x & 63) == 0)
        for (int j = 0; j < 3; ++j) red[j][threadIdx.x >> 6] = t[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < 3; ++j) {
            t[j] = 0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t[j] += red[j][k];
            out[j] = t[j];
        }
        out[3] = n - t[0] - t[1] - t[2];
    }
}

// ---------------------------------------------------------------------------
// tile routing
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_route_state(const float* __restrict__ z, long n, float z_lo,
                                                     float z_hi, uint8_t* __restrict__ st) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float v = z[i];
        st[i] = v < z_lo ? 0 : (v > z_hi ? 1 : 2);  // NaN logits take the exact path
    }
}

// Confident tiles of a routed frame take their state (0 or 1) in every mask
// byte; exact tiles (state 2) keep what the exact path wrote there.  One
// thread per 16-pixel row segment of a tile (consecutive threads: adjacent
// segments of one row).
__global__ __launch_bounds__(256) void k_route_apply(const uint8_t* __restrict__ state, int n_views, int H, int W,
                                                     int tiles_y, int tiles_x, uint8_t* __restrict__ M) {
    const long n = (long)n_views * H * tiles_x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int tx = (int)(i % tiles_x);
        const long vy = i / tiles_x;
        const int y = (int)(vy % H), v = (int)(vy / H);
        const uint8_t s = state[((size_t)v * tiles_y + y / kTile) * tiles_x + tx];
        if (s == 2) continue;
        uint8_t* row = M + ((size_t)v * H + y) * W;
        const int x0 = tx * kTile, x1 = min(x0 + kTile, W);
        if (x1 - x0 == kTile && (reinterpret_cast<uintptr_t>(row + x0) & 15) == 0) {
            const uint32_t w = s ? 0x01010101u : 0u;
            *reinterpret_cast<uint4*>(row + x0) = make_uint4(w, w, w, w);
        } else {
            for (int x = x0; x < x1; ++x) row[x] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// forward-warping ground truth (z-buffer) for the quality counts of Eq. (7)
// ---------------------------------------------------------------------------
// Pixel p = (x, y) lands at the nearest pixel of p - r*D(p)*u: t = r*D(p),
// tx = rint(x - t*c), ty = rint(y - t*s) (fp32, half to even).  Per view the
// targets live in a grid padded by `pad` pixels on every side (pad exceeds
// r * max|D|, so every target fits); the grid holds the largest disparity
// per target as an order-preserving uint32 (0 = nothing landed).
struct ZViews {
    float c[OCCL_MAX_VIEWS], s[OCCL_MAX_VIEWS], r[OCCL_MAX_VIEWS];
    int pad[OCCL_MAX_VIEWS];
    long long off[OCCL_MAX_VIEWS + 1];  // first grid cell of view v
};

__device__ __forceinline__ long long ztarget(const ZViews& zv, int v, int x, int y, float d, int H,
                                             int W) {
    const float t = __fmul_rn(zv.r[v], d);
    const int tx = (int)rintf(__fsub_rn((float)x, __fmul_rn(t, zv.c[v])));
    const int ty = (int)rintf(__fsub_rn((float)y, __fmul_rn(t, zv.s[v])));
    const int p = zv.pad[v];
    const int gw = W + 2 * p, gh = H + 2 * p;
    const int gx = tx + p, gy = ty + p;
    if (gx < 0 || gx >= gw || gy < 0 || gy >= gh) return -1;  // cannot happen for a finite D
    return zv.off[v] + (long long)gy * gw + gx;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_zbuf_splat(const float* __restrict__ D, int H, int W, int n_views,
                                                    ZViews zv, uint32_t* __restrict__ best) {
    const long long HW = (long long)H * W;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < HW * n_views;
         i += (long long)gridDim.x * blockDim.x) {
        const int v = (int)(i / HW);
        const long long k = i % HW;
        const int y = (int)(k / W), x = (int)(k % W);
        const float d = D[k];
        const long long g = ztarget(zv, v, x, y, d, H, W);
        if (g >= 0) atomicMax(&best[g], ford(d));
    }
}

__global__ __launch_bounds__(256) void k_zbuf_mark(const float* __restrict__ D, int H, int W, int n_views,
                                                   ZViews zv, float beta, const uint32_t* __restrict__ best,
                                                   uint8_t* __restrict__ M) {
    const long long HW = (long long)H * W;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < HW * n_views;
         i += (long long)gridDim.x * blockDim.x) {
        const int v = (int)(i / HW);
        const long long k = i % HW;
        const int y = (int)(k / W), x = (int)(k % W);
        const float d = D[k];
        const long long g = ztarget(zv, v, x, y, d, H, W);
        uint8_t m = 0;
        if (g >= 0) {
            const uint32_t o = best[g];
            const float b = __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
            m = __fsub_rn(b, d) > beta ? 1 : 0;
        }
        M[i] = m;
    }
}

// ---------------------------------------------------------------------------
// pixel-wise median fusion of K per-view disparity maps (NaN = no value)
// ---------------------------------------------------------------------------
// Per pixel the K values sit in registers; NaN becomes +inf and is not
// counted; an odd-even transposition network (K rounds) sorts them; the
// median of the first m = count(non-NaN) is picked with compile-time selects
// (an even m averages the two middle values: (a + b) * 0.5).
template <int K>
__global__ __launch_bounds__(256) void k_median_fuse(const float* __restrict__ maps, long long n,
                                                     float* __restrict__ D) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float v[K];
        int m = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float x = maps[(size_t)k * n + i];
            const bool ok = !isnan(x);
            v[k] = ok ? x : INFINITY;
            m += ok ? 1 : 0;
        }
#pragma unroll
        for (int round = 0; round < K; ++round)
#pragma unroll
            for (int k = round & 1; k + 1 < K; k += 2) {
                const float a = v[k], b = v[k + 1];
                v[k] = fminf(a, b);
                v[k + 1] = fmaxf(a, b);
            }
        float lo = 0.0f, hi = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            lo = (k == (m - 1) / 2) ? v[k] : lo;
            hi = (k == m / 2) ? v[k] : hi;
        }
        D[i] = m == 0 ? __int_as_float(0x7fc00000) : ((m & 1) ? hi : __fmul_rn(__fadd_rn(lo, hi), 0.5f));
    }
}

inline int grid_for(size_t n, int per_block, int cap) {
    size_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_scan_stats(hipStream_t st, const float* D, size_t n, uint32_t* dev) {
    // dev: 3 results, then room for kStatsBlocks * 3 partials
    const int nb = grid_for(n, 256 * 8, kStatsBlocks);
    hipLaunchKernelGGL(k_stats, dim3(nb), dim3(256), 0, st, D, n, dev + 3);
    hipLaunchKernelGGL(k_stats_sum, dim3(1), dim3(256), 0, st, dev + 3, nb, dev);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t st, uint32_t* p, long long n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((size_t)n, 256, 1024)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_edges_out(hipStream_t st, const float* D, int H, int W, float* E, float* A) {
    const size_t n = (size_t)H * W;
    hipLaunchKernelGGL(k_edges_out, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, D, H, W, E, A);
    return hipGetLastError();
}

hipError_t launch_route_state(hipStream_t st, const float* logits, size_t n, float z_lo, float z_hi,
                              uint8_t* tstate) {
    hipLaunchKernelGGL(k_route_state, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, logits, (long)n, z_lo, z_hi,
                       tstate);
    return hipGetLastError();
}

hipError_t launch_route_apply(hipStream_t st, const uint8_t* tstate, int n_views, int H, int W, int tiles_y,
                              int tiles_x, uint8_t* M) {
    const size_t n = (size_t)n_views * H * tiles_x;
    hipLaunchKernelGGL(k_route_apply, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, tstate, n_views, H, W,
                       tiles_y, tiles_x, M);
    return hipGetLastError();
}

long long zbuffer_cells(int H, int W, int n_views, const float* ratios, float max_abs_d) {
    long long n = 0;
    for (int v = 0; v < n_views; ++v) {
        const int pad = (int)std::ceil((double)ratios[v] * (double)max_abs_d) + 2;
        n += (long long)(H + 2 * pad) * (W + 2 * pad);
    }
    return n;
}

hipError_t launch_zbuffer(hipStream_t st, const float* D, int H, int W, int n_views, const ViewTable& vt,
                          float max_abs_d, float beta, uint32_t* best, uint8_t* M) {
    ZViews zv{};
    long long off = 0;
    for (int v = 0; v < n_views; ++v) {
        zv.c[v] = vt.c[v];
        zv.s[v] = vt.s[v];
        zv.r[v] = vt.r[v];
        zv.pad[v] = (int)std::ceil((double)vt.r[v] * (double)max_abs_d) + 2;
        zv.off[v] = off;
        off += (long long)(H + 2 * zv.pad[v]) * (W + 2 * zv.pad[v]);
    }
    zv.off[n_views] = off;
    const size_t n = (size_t)H * W * n_views;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((size_t)off, 256, 8192)), dim3(256), 0, st, best, off);
    hipLaunchKernelGGL(k_zbuf_splat, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, D, H, W, n_views, zv, best);
    hipLaunchKernelGGL(k_zbuf_mark, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, D, H, W, n_views, zv, beta,
                       best, M);
    return hipGetLastError();
}

hipError_t launch_median_fuse(hipStream_t st, const float* maps, int K, long long n, float* D) {
    const dim3 grid(grid_for((size_t)n, 256, 8192)), block(256);
    switch (K) {
#define OCCL_MEDIAN_CASE(k) \
    case k: hipLaunchKernelGGL(k_median_fuse<k>, grid, block, 0, st, maps, n, D); break;
        OCCL_MEDIAN_CASE(1) OCCL_MEDIAN_CASE(2) OCCL_MEDIAN_CASE(3) OCCL_MEDIAN_CASE(4)
        OCCL_MEDIAN_CASE(5) OCCL_MEDIAN_CASE(6) OCCL_MEDIAN_CASE(7) OCCL_MEDIAN_CASE(8)
        OCCL_MEDIAN_CASE(9) OCCL_MEDIAN_CASE(10) OCCL_MEDIAN_CASE(11) OCCL_MEDIAN_CASE(12)
        OCCL_MEDIAN_CASE(13) OCCL_MEDIAN_CASE(14) OCCL_MEDIAN_CASE(15) OCCL_MEDIAN_CASE(16)
#undef OCCL_MEDIAN_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_confusion(hipStream_t st, const uint8_t* pred, const uint8_t* ref, size_t n,
                            unsigned long long* dev4) {
    // dev4: 4 results, then room for kConfusionBlocks * 3 partials
    const int nb = grid_for(n, 256 * 16 * 4, kConfusionBlocks);
    hipLaunchKernelGGL(k_confusion, dim3(nb), dim3(256), 0, st, pred, ref, n, dev4 + 4);
    hipLaunchKernelGGL(k_confusion_sum, dim3(1), dim3(256), 0, st, dev4 + 4, nb, n, dev4);
    return hipGetLastError();
}

}  // namespace occl
