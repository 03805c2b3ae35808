// k_cnn.hip -- gfx950 kernels of the learned tile proposal: a 6-layer 3x3
// convolutional network (8->32 s2, 32->32 s2, 32->32 s2, 32->32 s2,
// 32->32 s1, 32->1 s1; ReLU after all but the last) in BF16 with FP32
// accumulation, trained and run on MFMA.
//
// Layouts: activations NHWC bf16 [N][H][W][C]; weights [Cout][3][3][Cin]
// (bf16 copy of fp32 master weights), biases fp32; logits fp32 [N][Ht][Wt].
// Output size of a stride-s layer: ceil(H / s).
//
// The 32-output-channel layers are implicit GEMMs on MFMA: one wavefront
// computes 32 output pixels x 32 channels on v_mfma_f32_32x32x16_bf16
// (operand layout checked on the device): lane l supplies
// A[l % 32][8*(l/32) + i] and B[8*(l/32) + i][l % 32], i = 0..7, and
// accumulator register j of lane l holds D[8*(j/4) + 4*(l/32) + (j%4)][l % 32].
//   forward  M = output pixels, N = output channels, K = 9 * Cin (32x32x16;
//            weights resident in registers, persistent wavefronts)
//   dgrad    M = input pixels,  N = input channels,  K = 9 * Cout (weights
//            pre-transposed to [tap][Cin][Cout]; invalid taps of a strided
//            layer contribute zeros)
//   wgrad    M = output channels, N = (tap, Cin) columns, K = pixels; split
//            over pixel chunks into FP32 partials that a second kernel sums
//            in a fixed order (deterministic)
// The 1-channel last layer and the loss use plain VALU kernels.
#include <algorithm>

#include "occl_cnn.h"

namespace occl {
namespace {

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Pixels per weight-gradient partial (one block of k_conv_wgrad), and per
// partial of the last layer's (one block of k_wgrad_last).
constexpr int kWgradChunk = 256;
constexpr int kWgradStep = 32;  // pixels staged per step of k_conv_wgrad (a multiple of 16 dividing kWgradChunk)
constexpr int kLastChunk = 32;

// D += A B on v_mfma_f32_32x32x16_bf16 (lane layout in the header comment)
__device__ __forceinline__ f32x16 mfma16(s16x8 a, s16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}


// fp32 -> bf16, round to nearest, ties to even: gfx950's v_cvt_pk_bf16_f32
// (checked on the device against the integer rounding rule on 2^25 bit
// patterns, every finite value class included)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// The forward kernels run the MFMA with the weights as A (rows = output
// channels) and the pixels as B, so accumulator register 4 g + i of lane l
// holds output channel 8 g + 4 (l / 32) + i of pixel l % 32: a lane owns 16
// channels of one pixel, in four runs of 4.  relu_pack turns run g into 4
// bf16 (bias added, ReLU).
__device__ __forceinline__ uint2 relu_pack(const f32x16& acc, const float (&bias)[16], int g) {
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float x = acc[4 * g + i] + bias[4 * g + i];
        v[i] = x > 0.0f ? x : 0.0f;
    }
    return uint2{pk_bf16(v[0], v[1]), pk_bf16(v[2], v[3])};
}

__device__ __forceinline__ void load_bias16(const float* __restrict__ b, int q, float (&out)[16]) {
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[4 * g + i] = b[8 * g + 4 * q + i];
}

// ---------------------------------------------------------------------------
// input pack: per view, D * r / L, E / 8, cos A, sin A, cos alpha, sin alpha,
// r / 2, 0 (A = atan2(E_y, E_x) of the forward-difference edge maps)
// ---------------------------------------------------------------------------
struct PackViews {
    float c[OCCL_MAX_VIEWS], s[OCCL_MAX_VIEWS], r[OCCL_MAX_VIEWS], inv_L[OCCL_MAX_VIEWS];
};

__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ D, int H, int W, int n_views,
                                              PackViews pv, uint16_t* __restrict__ X) {
    const size_t HW = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i % W);
        const float d = D[i];
        const float ex = (x + 1 < W) ? D[i + 1] - d : 0.0f;
        const float ey = (y + 1 < H) ? D[i + W] - d : 0.0f;
        const float E = sqrtf(ex * ex + ey * ey);
        const float ca = E > 0.0f ? ex / E : 1.0f;
        const float sa = E > 0.0f ? ey / E : 0.0f;
        for (int v = 0; v < n_views; ++v) {
            uint16_t o[8];
            o[0] = f2bf(d * pv.r[v] * pv.inv_L[v]);
            o[1] = f2bf(E * 0.125f);
            o[2] = f2bf(ca);
            o[3] = f2bf(sa);
            o[4] = f2bf(pv.c[v]);
            o[5] = f2bf(pv.s[v]);
            o[6] = f2bf(pv.r[v] * 0.5f);
            o[7] = 0;
            uint4 q;
            q.x = o[0] | ((uint32_t)o[1] << 16);
            q.y = o[2] | ((uint32_t)o[3] << 16);
            q.z = o[4] | ((uint32_t)o[5] << 16);
            q.w = o[6] | ((uint32_t)o[7] << 16);
            *reinterpret_cast<uint4*>(X + ((size_t)v * HW + i) * 8) = q;
        }
    }
}

// The view-independent part of the input, once per frame: G[i] = {D (fp32
// bits), bf16 E/8, bf16 cos A | bf16 sin A << 16, 0}, computed exactly as
// k_pack computes those channels.
__global__ __launch_bounds__(256) void k_pack_base(const float* __restrict__ D, int H, int W,
                                                   uint4* __restrict__ G) {
    const size_t HW = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i % W);
        const float d = D[i];
        const float ex = (x + 1 < W) ? D[i + 1] - d : 0.0f;
        const float ey = (y + 1 < H) ? D[i + W] - d : 0.0f;
        const float E = sqrtf(ex * ex + ey * ey);
        const float ca = E > 0.0f ? ex / E : 1.0f;
        const float sa = E > 0.0f ? ey / E : 0.0f;
        G[i] = uint4{__float_as_uint(d), (uint32_t)f2bf(E * 0.125f),
                     (uint32_t)f2bf(ca) | ((uint32_t)f2bf(sa) << 16), 0u};
    }
}

// First layer (8 -> 32, stride 2) of every view straight from G: the packed
// input of view v at a tap pixel is {bf16(D r / L), E/8, cos A, sin A,
// cos alpha, sin alpha, r/2, 0} (bit-identical to k_pack's), assembled in
// registers, so the 16-byte-per-pixel-per-view input never goes to memory.
// Each wavefront loads a tile's G values once and runs the MFMA chain of
// every view on them.  Output NHWC bf16 [n_views][Ho][Wo][32].
__global__ __launch_bounds__(256) void k_conv0_fused(const uint4* __restrict__ G, int H, int W,
                                                     int n_views, PackViews pv,
                                                     const uint16_t* __restrict__ Wt,
                                                     const float* __restrict__ bias,
                                                     uint16_t* __restrict__ Y, int Ho, int Wo) {
    constexpr int CIN = 8, NS = 5;
    __shared__ s16x8 wl[NS * 2 * 32];
    for (int i = threadIdx.x; i < NS * 64; i += blockDim.x) {
        const int st = i / 64, qq = (i / 32) % 2, co = i % 32;
        const int tap = 2 * st + qq;
        wl[i] = tap < 9 ? *reinterpret_cast<const s16x8*>(Wt + ((size_t)co * 9 + tap) * CIN)
                        : s16x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int q = lane >> 5, i32 = lane & 31;
    float bv[16];
    load_bias16(bias, q, bv);
    const long total = (long)Ho * Wo;  // per view
    const long ntiles = (total + 31) / 32;
    const long step = (long)gridDim.x * (blockDim.x >> 6);
    for (long tile = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntiles; tile += step) {
        const long p = tile * 32 + i32;
        const bool pvalid = p < total;
        const int oy = pvalid ? (int)(p / Wo) : 0, ox = pvalid ? (int)(p % Wo) : 0;
        uint4 g[NS];
        bool in[NS];
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const int tap = 2 * st + q;
            const int iy = oy * 2 + tap / 3 - 1, ix = ox * 2 + tap % 3 - 1;
            in[st] = pvalid && tap < 9 && iy >= 0 && iy < H && ix >= 0 && ix < W;
            g[st] = in[st] ? G[(size_t)iy * W + ix] : uint4{0u, 0u, 0u, 0u};
        }
        for (int v = 0; v < n_views; ++v) {
            const float r = pv.r[v], il = pv.inv_L[v];
            const uint32_t w2 = (uint32_t)f2bf(pv.c[v]) | ((uint32_t)f2bf(pv.s[v]) << 16);
            const uint32_t w3 = (uint32_t)f2bf(r * 0.5f);
            int z;
            asm volatile("s_mov_b32 %0, 0" : "=s"(z));
            f32x16 acc = {};
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                const uint32_t ch0 = f2bf(__uint_as_float(g[st].x) * r * il);
                const uint4 w = in[st] ? uint4{ch0 | (g[st].y << 16), g[st].z, w2, w3} : uint4{0u, 0u, 0u, 0u};
                acc = mfma16(wl[st * 64 + lane + z], __builtin_bit_cast(s16x8, w), acc);
            }
            if (pvalid) {
                uint16_t* yp = Y + ((size_t)v * total + p) * 32 + 4 * q;
#pragma unroll
                for (int g = 0; g < 4; ++g) *reinterpret_cast<uint2*>(yp + 8 * g) = relu_pack(acc, bv, g);
            }
        }
    }
}

// Layers 0 and 1 of every view fused, straight from G.  A block owns an
// output tile of layer 1 (TY rows x 32 columns).  It stages the G values
// under the tile (4 TY + 3 rows x 131 columns) in LDS once for all views;
// per view it computes the layer-0 outputs under the tile (2 TY + 1 rows x
// 65 columns, zero outside the layer-0 image) into LDS, then layer 1 from
// LDS, so layer 0's output (the largest tensor of the network) never goes to
// memory.  The layer-0 tile is stored by column parity ([row][parity]
// [column / 2][32 channels]), so the stride-2 taps of layer 1 read
// consecutive entries across lanes (entries padded to 80 bytes to spread
// the LDS banks).  Layer-1 weights stay in
// registers for all views of the tile, layer-0 weights in LDS.  The
// arithmetic (K order, roundings) is that of k_conv0_fused followed by
// k_conv_fwd_p<32, 2>, so the result is identical.
template <int TY>
__global__ __launch_bounds__(64 * TY) void k_conv01_fused(
    const uint4* __restrict__ G, int H, int W, int n_views, PackViews pv,
    const uint16_t* __restrict__ W0, const float* __restrict__ b0, const uint16_t* __restrict__ W1,
    const float* __restrict__ b1, uint16_t* __restrict__ Y1, int H0, int W0n, int H1, int W1n) {
    constexpr int TX = 32;
    constexpr int R0 = 2 * TY + 1, C0 = 2 * TX + 1;
    constexpr int CE = TX + 1;        // entries per (row, parity)
    constexpr int NP0 = R0 * C0;      // layer-0 pixels of the tile
    constexpr int NT0 = (NP0 + 31) / 32;
    constexpr int RG = 2 * R0 + 1, CG = 2 * C0 + 1;  // G window
    constexpr int ES = 40;            // entry stride in bf16: 80 bytes, an odd number of 16-byte
                                      // slots, so neighbouring entries fall on different banks
    __shared__ uint16_t l0[R0 * 2 * CE * ES];
    __shared__ float gsd[RG * CG];    // D of the G window
    __shared__ uint2 gse[RG * CG];    // {E/8, cos A | sin A << 16} of the G window
    __shared__ s16x8 wl0[5 * 64];
    for (int i = threadIdx.x; i < 5 * 64; i += blockDim.x) {
        const int st = i / 64, qq = (i / 32) % 2, co = i % 32;
        const int tap = 2 * st + qq;
        wl0[i] = tap < 9 ? *reinterpret_cast<const s16x8*>(W0 + ((size_t)co * 9 + tap) * 8)
                         : s16x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int q = lane >> 5, i32 = lane & 31;
    s16x8 bw[18];
#pragma unroll
    for (int st = 0; st < 18; ++st) {
        const int k0 = 16 * st + 8 * q;
        bw[st] = *reinterpret_cast<const s16x8*>(W1 + ((size_t)i32 * 9 + k0 / 32) * 32 + k0 % 32);
    }
    float bv0[16], bv1[16];
    load_bias16(b0, q, bv0);
    load_bias16(b1, q, bv1);
    const int tiles_x = (W1n + TX - 1) / TX, tiles_y = (H1 + TY - 1) / TY;
    for (int tile = blockIdx.x; tile < tiles_x * tiles_y; tile += gridDim.x) {
        const int Ya = (tile / tiles_x) * TY, Xa = (tile % tiles_x) * TX;
        const int gy0 = 2 * Ya - 1, gx0 = 2 * Xa - 1;  // layer-0 coordinates of the tile's (0, 0)
        const int dy0 = 2 * gy0 - 1, dx0 = 2 * gx0 - 1;  // frame coordinates of the G window's (0, 0)
        __syncthreads();  // the previous tile's readers of gs are done
        for (int i = threadIdx.x; i < RG * CG; i += blockDim.x) {
            const int iy = dy0 + i / CG, ix = dx0 + i % CG;
            const uint4 g = (iy >= 0 && iy < H && ix >= 0 && ix < W) ? G[(size_t)iy * W + ix]
                                                                     : uint4{0u, 0u, 0u, 0u};
            gsd[i] = __uint_as_float(g.x);
            gse[i] = uint2{g.y, g.z};
        }
        __syncthreads();
        for (int v = 0; v < n_views; ++v) {
            const float r = pv.r[v], il = pv.inv_L[v];
            const uint32_t w2 = (uint32_t)f2bf(pv.c[v]) | ((uint32_t)f2bf(pv.s[v]) << 16);
            const uint32_t w3 = (uint32_t)f2bf(r * 0.5f);
            // ---- layer 0 into LDS ----
            // Out-of-frame G entries are zero, so channels 0-3 of an outside tap
            // are already 0 and only the constant channels need masking; tap 9
            // (K padding) has zero weights and reads any in-window entry.
            for (int t0 = wave; t0 < NT0; t0 += TY) {
                const int p = t0 * 32 + i32;
                const int pc = p < NP0 ? p : NP0 - 1;
                const int r0 = pc / C0, c0 = pc % C0;
                const int gy = gy0 + r0, gx = gx0 + c0;
                const bool inimg = p < NP0 && gy >= 0 && gy < H0 && gx >= 0 && gx < W0n;
                const int fy = 2 * gy - 1, fx = 2 * gx - 1;  // frame coordinates of tap (0, 0)
                bool rok[3], cok[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    rok[k] = fy + k >= 0 && fy + k < H;
                    cok[k] = fx + k >= 0 && fx + k < W;
                }
                const int gbase = 2 * r0 * CG + 2 * c0;
                int z;
                asm volatile("s_mov_b32 %0, 0" : "=s"(z));
                f32x16 acc = {};
#pragma unroll
                for (int st = 0; st < 5; ++st) {
                    const int ta = 2 * st, tb = 2 * st + 1 < 9 ? 2 * st + 1 : 0;  // lane half 0 / 1
                    const int gi = gbase + (q ? (tb / 3) * CG + tb % 3 : (ta / 3) * CG + ta % 3);
                    const bool in = q ? (2 * st + 1 < 9 && rok[tb / 3] && cok[tb % 3])
                                      : (rok[ta / 3] && cok[ta % 3]);
                    const uint2 ge = gse[gi];
                    const uint32_t ch0 = f2bf(gsd[gi] * r * il);
                    const uint4 w = uint4{ch0 | (ge.x << 16), ge.y, in ? w2 : 0u, in ? w3 : 0u};
                    acc = mfma16(wl0[st * 64 + lane + z], __builtin_bit_cast(s16x8, w), acc);
                }
                if (p < NP0) {
                    // this lane's pixel (r0, c0): 16 channels, zero outside the layer-0 image
                    uint16_t* dst = l0 + ((r0 * 2 + (c0 & 1)) * CE + (c0 >> 1)) * ES + 4 * q;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const uint2 v2 = relu_pack(acc, bv0, g);
                        *reinterpret_cast<uint2*>(dst + 8 * g) = inimg ? v2 : uint2{0u, 0u};
                    }
                }
            }
            __syncthreads();
            // ---- layer 1 from LDS: wavefront `wave` takes output row Ya + wave ----
            {
                const int ly = wave, lx = i32;
                int z;
                asm volatile("s_mov_b32 %0, 0" : "=s"(z));
                // lane base (column lx, channel half q) + a per-step constant
                const uint16_t* lb = l0 + (2 * ly * 2 * CE + lx) * ES + 8 * q + z;
                f32x16 acc = {};
#pragma unroll
                for (int st = 0; st < 18; ++st) {
                    const int tap = st / 2, ky = tap / 3, kx = tap % 3;
                    const int off = ((ky * 2 + (kx & 1)) * CE + (kx >> 1)) * ES + 16 * (st % 2);
                    acc = mfma16(bw[st], *reinterpret_cast<const s16x8*>(lb + off), acc);
                }
                const int Yo = Ya + ly, xo = Xa + lx;
                if (Yo < H1 && xo < W1n) {
                    uint16_t* yp = Y1 + (((size_t)v * H1 + Yo) * W1n + xo) * 32 + 4 * q;
#pragma unroll
                    for (int g = 0; g < 4; ++g) *reinterpret_cast<uint2*>(yp + 8 * g) = relu_pack(acc, bv1, g);
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// forward, 32 output channels, bias + ReLU (MFMA implicit GEMM)
// ---------------------------------------------------------------------------
// Forward of a 32-output-channel layer, persistent: the block stages the B
// operand of all K steps (the whole weight tensor, K = 9 * CIN padded to a
// multiple of 16) in LDS once, laid out so that a K step's fragment is one
// conflict-free 16-byte read per lane; every wavefront then walks 32-pixel
// tiles, issuing all A loads of a tile (one 16-byte NHWC load per lane per K
// step) before its MFMA chain, then bias + ReLU + bf16.  K index
// k = tap * CIN + ci; a K step of 16 is tap k0 / CIN, channels k0 % CIN .. +7
// for k0 = 16 s + 8 (l / 32).
template <int CIN, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_conv_fwd_p(const uint16_t* __restrict__ X,
                                                    const uint16_t* __restrict__ Wt,
                                                    const float* __restrict__ bias,
                                                    uint16_t* __restrict__ Y, int N, int H, int W,
                                                    int Ho, int Wo) {
    constexpr int NS = (9 * CIN + 15) / 16;
    __shared__ s16x8 wl[NS * 2 * 32];  // [step][lane half][output channel]
    for (int i = threadIdx.x; i < NS * 64; i += blockDim.x) {
        const int st = i / 64, qq = (i / 32) % 2, co = i % 32;
        const int k0 = 16 * st + 8 * qq;
        const int tap = k0 / CIN, coff = k0 % CIN;
        wl[i] = tap < 9 ? *reinterpret_cast<const s16x8*>(Wt + ((size_t)co * 9 + tap) * CIN + coff)
                        : s16x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int q = lane >> 5, i32 = lane & 31;
    float bv[16];
    load_bias16(bias, q, bv);
    const long total = (long)N * Ho * Wo;
    const long ntiles = (total + 31) / 32;
    const long step = (long)gridDim.x * (blockDim.x >> 6);
    for (long tile = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntiles; tile += step) {
        const long p = tile * 32 + i32;  // this lane's pixel
        const bool pv = p < total;
        const int n = pv ? (int)(p / ((long)Ho * Wo)) : 0;
        const int rem = pv ? (int)(p % ((long)Ho * Wo)) : 0;
        const int oy = rem / Wo, ox = rem % Wo;
        s16x8 a[NS];
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const int k0 = 16 * st + 8 * q;
            const int tap = k0 / CIN, coff = k0 % CIN;
            const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
            const bool in = pv && tap < 9 && iy >= 0 && iy < H && ix >= 0 && ix < W;
            a[st] = in ? *reinterpret_cast<const s16x8*>(X + (((size_t)n * H + iy) * W + ix) * CIN + coff)
                       : s16x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
        // an opaque zero keeps the weight reads inside the loop (hoisted, they
        // would hold 72 registers and halve the resident wavefronts)
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        f32x16 acc = {};
#pragma unroll
        for (int st = 0; st < NS; ++st) acc = mfma16(wl[st * 64 + lane + z], a[st], acc);
        if (pv) {
            uint16_t* yp = Y + p * 32 + 4 * q;
#pragma unroll
            for (int g = 0; g < 4; ++g) *reinterpret_cast<uint2*>(yp + 8 * g) = relu_pack(acc, bv, g);
        }
    }
}

// last layer: 32 -> 1, stride 1, no activation, fp32 logits
__global__ __launch_bounds__(256) void k_conv_last(const uint16_t* __restrict__ X,
                                                   const uint16_t* __restrict__ Wt,
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ Z, int N, int H, int W) {
    const long total = (long)N * H * W;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (long)gridDim.x * blockDim.x) {
        const int n = (int)(p / ((long)H * W));
        const int rem = (int)(p % ((long)H * W));
        const int oy = rem / W, ox = rem % W;
        float acc = bias[0];
        for (int t = 0; t < 9; ++t) {
            const int iy = oy + t / 3 - 1, ix = ox + t % 3 - 1;
            if (iy < 0 || iy >= H || ix < 0 || ix >= W) continue;
            const uint16_t* xr = X + (((size_t)n * H + iy) * W + ix) * 32;
            const uint16_t* wr = Wt + t * 32;
            for (int ci = 0; ci < 32; ++ci) acc += bf2f(xr[ci]) * bf2f(wr[ci]);
        }
        Z[p] = acc;
    }
}

// ---------------------------------------------------------------------------
// loss: soft binary cross-entropy on the logits, mean over all tiles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ Z, const float* __restrict__ T,
                                             float* __restrict__ dZ, double* __restrict__ partial,
                                             long n) {
    __shared__ double red[256];
    double acc = 0.0;
    const float inv = 1.0f / (float)n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const float z = Z[i], t = T[i];
        const float sg = 1.0f / (1.0f + expf(-z));
        dZ[i] = (sg - t) * inv;
        acc += (double)(fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))) - t * z);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// backward of the last layer (32 -> 1, stride 1)
// ---------------------------------------------------------------------------
// dX[n][y][x][ci] = sum_t dZ[n][y - ky + 1][x - kx + 1] * w[t][ci]  -> bf16
__global__ __launch_bounds__(256) void k_dgrad_last(const float* __restrict__ dZ,
                                                    const uint16_t* __restrict__ Wt,
                                                    uint16_t* __restrict__ dX, int N, int H, int W) {
    const long total = (long)N * H * W * 32;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long)gridDim.x * blockDim.x) {
        const int ci = (int)(i & 31);
        const long p = i >> 5;
        const int n = (int)(p / ((long)H * W));
        const int rem = (int)(p % ((long)H * W));
        const int y = rem / W, x = rem % W;
        float acc = 0.0f;
        for (int t = 0; t < 9; ++t) {
            const int oy = y - t / 3 + 1, ox = x - t % 3 + 1;
            if (oy < 0 || oy >= H || ox < 0 || ox >= W) continue;
            acc += dZ[((size_t)n * H + oy) * W + ox] * bf2f(Wt[t * 32 + ci]);
        }
        dX[i] = f2bf(acc);
    }
}

// partial sums over pixel chunks of dW[t][ci] = sum_p dZ[p] X[in(p, t)][ci]
// and db = sum_p dZ[p]: block b handles chunk b, thread k column k (288 + 1)
__global__ __launch_bounds__(320) void k_wgrad_last(const float* __restrict__ dZ,
                                                    const uint16_t* __restrict__ X,
                                                    float* __restrict__ partial, int N, int H, int W,
                                                    int chunk) {
    const int k = threadIdx.x;
    if (k > 288) return;
    const long total = (long)N * H * W;
    const long p0 = (long)blockIdx.x * chunk;
    const long p1 = p0 + chunk < total ? p0 + chunk : total;
    float acc = 0.0f;
    const int t = k / 32, ci = k % 32;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    // the chunk's first pixel by division, the others by stepping along the row
    const long hw = (long)H * W;
    int n = (int)(p0 / hw);
    const int rem = (int)(p0 - (long)n * hw);
    int y = rem / W, x = rem - y * W;
    for (long p = p0; p < p1; ++p) {
        const float g = dZ[p];
        if (k == 288) {
            acc += g;
        } else {
            const int iy = y + dy, ix = x + dx;
            if (iy >= 0 && iy < H && ix >= 0 && ix < W)
                acc += g * bf2f(X[(((size_t)n * H + iy) * W + ix) * 32 + ci]);
        }
        if (++x == W) {
            x = 0;
            if (++y == H) {
                y = 0;
                ++n;
            }
        }
    }
    partial[(size_t)blockIdx.x * 289 + k] = acc;
}

// ---------------------------------------------------------------------------
// backward of a 32-output-channel layer with ReLU: g = dY * [Y > 0]
// ---------------------------------------------------------------------------
__device__ __forceinline__ s16x8 relu_grad8(const uint16_t* dy, const uint16_t* y) {
    const s16x8 g = *reinterpret_cast<const s16x8*>(dy), a = *reinterpret_cast<const s16x8*>(y);
    s16x8 o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = (bf2f((uint16_t)a[i]) > 0.0f) ? g[i] : (short)0;
    return o;
}

// dX (bf16 [N][H][W][32]) of a layer with CIN = 32 input channels; WT is the
// weight transposed to [tap][ci][co].
template <int S>
__global__ __launch_bounds__(256) void k_conv_dgrad(const uint16_t* __restrict__ dY,
                                                    const uint16_t* __restrict__ Y,
                                                    const uint16_t* __restrict__ WT,
                                                    uint16_t* __restrict__ dX, int N, int H, int W,
                                                    int Ho, int Wo) {
    const int lane = threadIdx.x & 63;
    const int q = lane >> 5, i32 = lane & 31;
    const long total = (long)N * H * W;
    const long m0 = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
    if (m0 >= total) return;
    const long p = m0 + i32;
    const bool pv = p < total;
    const int n = pv ? (int)(p / ((long)H * W)) : 0;
    const int rem = pv ? (int)(p % ((long)H * W)) : 0;
    const int iy = rem / W, ix = rem % W;
    f32x16 acc = {};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ny = iy + 1 - t / 3, nx = ix + 1 - t % 3;  // = oy * S, ox * S
        const int oy = ny / S, ox = nx / S;
        const bool ok = pv && ny >= 0 && nx >= 0 && (ny % S) == 0 && (nx % S) == 0 && oy < Ho && ox < Wo;
        // a tap under which no pixel of the wavefront has an output adds
        // nothing (with stride 2, 3 or 6 of the 9 taps of a row's pixels)
        if (__ballot(ok) == 0) continue;  // uniform
        const size_t o = (((size_t)n * Ho + (ok ? oy : 0)) * Wo + (ok ? ox : 0)) * 32;
        const uint16_t* wrow = WT + ((size_t)t * 32 + i32) * 32;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {  // output channels 16 cc .. 16 cc + 15 (8 per lane half)
            const s16x8 a = ok ? relu_grad8(dY + o + 16 * cc + 8 * q, Y + o + 16 * cc + 8 * q)
                               : s16x8{0, 0, 0, 0, 0, 0, 0, 0};
            const s16x8 b = *reinterpret_cast<const s16x8*>(wrow + 16 * cc + 8 * q);
            acc = mfma16(a, b, acc);
        }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const long pr = m0 + 8 * (j / 4) + 4 * q + (j % 4);
        if (pr < total) dX[pr * 32 + i32] = f2bf(acc[j]);
    }
}

// wgrad partials of a 32-output-channel layer: block `chunk` computes every
// 32 x 32 tile of dW[co][t*CIN + ci] (co rows, columns col = t*CIN + ci) over
// the chunk's pixels; partial layout [chunk][32 * 9*CIN + 32]: dW, then the
// bias gradient's 32 (the layout of the layer's gradient).  Per step of
// kWgradStep pixels the block stages, with 16-byte loads, the relu-masked
// output gradient g = dY [Y > 0] (gs[pixel][co]) and the input under each tap
// (xs[pixel][col], zero outside the image) in LDS; wavefront w then runs the
// column tiles w, w + 4, ..., one MFMA per 16 pixels in pixel order, taking
// its operands from LDS (8 pixels of one row or column per lane half).  The
// bias gradient's partial is the sum of g over the chunk's pixels, per pixel
// slot in step order, then the slots in order.
template <int CIN, int S>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t* __restrict__ dY,
                                                    const uint16_t* __restrict__ Y,
                                                    const uint16_t* __restrict__ X,
                                                    float* __restrict__ partial, int N, int H, int W, int Ho,
                                                    int Wo, int chunk) {
    constexpr int NCOL = 9 * CIN;
    constexpr int NOUT = 32 * NCOL + 32;  // partial row: dW, then the bias
    constexpr int NT = (NCOL + 31) / 32;  // column tiles
    constexpr int NCP = NT * 32;          // columns, padded to whole tiles
    constexpr int TPW = (NT + 3) / 4;     // tiles per wavefront
    constexpr int XV = CIN / 8;           // 16-byte vectors of X per pixel
    constexpr int KS = kWgradStep;        // pixels per staged step (two MFMA K blocks of 16)
    __shared__ __align__(16) uint16_t gs[KS][32];
    __shared__ __align__(16) uint16_t xs[KS][NCP];
    __shared__ float bred[4 * KS][8];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int q = lane >> 5, i32 = lane & 31;
    const long total = (long)N * Ho * Wo;
    const long p0 = (long)blockIdx.x * chunk;
    const long hwo = (long)Ho * Wo;
    if constexpr (NCP > NCOL)  // the padding columns of the last tile stay zero
        for (int i = tid; i < KS * (NCP - NCOL); i += 256) xs[i / (NCP - NCOL)][NCOL + i % (NCP - NCOL)] = 0;
    f32x16 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = f32x16{};
    float bs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // threads < 4 KS: slot tid / 4, channels 8 (tid % 4) ..
    for (int k0 = 0; k0 < chunk; k0 += KS) {
        __syncthreads();    // the previous step's operands have been read
        if (tid < 4 * KS) {  // g: KS pixels x 4 vectors of 8 channels
            const int pi = tid >> 2, v = tid & 3;
            const long p = p0 + k0 + pi;
            s16x8 g = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (p < total && p < p0 + chunk) {
                const s16x8 d8 = *reinterpret_cast<const s16x8*>(dY + (size_t)p * 32 + 8 * v);
                const s16x8 y8 = *reinterpret_cast<const s16x8*>(Y + (size_t)p * 32 + 8 * v);
#pragma unroll
                for (int c = 0; c < 8; ++c) g[c] = (bf2f((uint16_t)y8[c]) > 0.0f) ? d8[c] : (short)0;
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) bs[c] += bf2f((uint16_t)g[c]);
            *reinterpret_cast<s16x8*>(&gs[pi][8 * v]) = g;
        }
        {  // x: KS pixels x 9 taps x XV vectors; this thread's pixel slot is tid % KS
            const int pi = tid % KS;
            const long p = p0 + k0 + pi;
            const bool pin = p < total && p < p0 + chunk;
            const long pc = pin ? p : 0;
            const int n = (int)(pc / hwo);
            const int rem = (int)(pc - (long)n * hwo);
            const int oy = rem / Wo, ox = rem - oy * Wo;
            for (int r = tid / KS; r < 9 * XV; r += 256 / KS) {
                const int t = r / XV, v = r % XV;
                const int iy = oy * S + t / 3 - 1, ix = ox * S + t % 3 - 1;
                s16x8 x = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
                if (pin && iy >= 0 && iy < H && ix >= 0 && ix < W)
                    x = *reinterpret_cast<const s16x8*>(X + (((size_t)n * H + iy) * W + ix) * CIN + 8 * v);
                *reinterpret_cast<s16x8*>(&xs[pi][t * CIN + 8 * v]) = x;
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < KS; h += 16) {  // pixels in order: the same MFMA sequence as 16-pixel steps
            s16x8 a;
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = (short)gs[h + 8 * q + i][i32];  // A[co = i32][pixel]
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int tile = wave + 4 * u;
                if (tile < NT) {  // uniform
                    s16x8 b;
#pragma unroll
                    for (int i = 0; i < 8; ++i) b[i] = (short)xs[h + 8 * q + i][tile * 32 + i32];  // B[pixel][col]
                    acc[u] = mfma16(a, b, acc[u]);
                }
            }
        }
    }
    if (tid < 4 * KS) {
#pragma unroll
        for (int c = 0; c < 8; ++c) bred[tid][c] = bs[c];
    }
    __syncthreads();
    if (tid < 32) {
        float sum = 0.0f;
        for (int pi = 0; pi < KS; ++pi) sum += bred[pi * 4 + tid / 8][tid % 8];
        partial[(size_t)blockIdx.x * NOUT + 32 * NCOL + tid] = sum;
    }
    float* out = partial + (size_t)blockIdx.x * NOUT;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int col = (wave + 4 * u) * 32 + i32;
        if (wave + 4 * u < NT && col < NCOL) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int co = 8 * (r / 4) + 4 * q + (r % 4);
                out[(size_t)co * NCOL + col] = acc[u][r];
            }
        }
    }
}

// Chunk partials partial[c][k] (c < n_chunks, k < n_out) are summed in a
// fixed order, so a gradient does not depend on the launch: with more than
// kReduceGroup chunks, first the chunks of each group of kReduceGroup in
// order, the sum written in place over the group's first chunk (block
// (x, g): group g), then those group sums in order.
constexpr int kReduceGroup = 64;
__global__ __launch_bounds__(256) void k_reduce_groups(float* __restrict__ partial, int n_chunks, int n_out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_out) return;
    const int c0 = (int)blockIdx.y * kReduceGroup;
    const int c1 = c0 + kReduceGroup < n_chunks ? c0 + kReduceGroup : n_chunks;
    float s = 0.0f;
#pragma unroll 8
    for (int c = c0; c < c1; ++c) s += partial[(size_t)c * n_out + k];  // loads in flight together, sums in order
    partial[(size_t)c0 * n_out + k] = s;
}

// out[k] = sum of partial[c][k] over c = 0, step, 2 step, ... < n_chunks, in order
__global__ __launch_bounds__(256) void k_reduce_chunks(const float* __restrict__ partial,
                                                       float* __restrict__ out, int n_chunks,
                                                       int n_out, int step) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_out) return;
    float s = 0.0f;
#pragma unroll 8
    for (int c = 0; c < n_chunks; c += step) s += partial[(size_t)c * n_out + k];
    out[k] = s;
}

void reduce_chunks(hipStream_t st, float* partial, float* out, int n_chunks, int n_out) {
    const int groups = (n_chunks + kReduceGroup - 1) / kReduceGroup;
    if (groups > 1)
        hipLaunchKernelGGL(k_reduce_groups, dim3((n_out + 255) / 256, groups), dim3(256), 0, st, partial, n_chunks,
                           n_out);
    hipLaunchKernelGGL(k_reduce_chunks, dim3((n_out + 255) / 256), dim3(256), 0, st, partial, out, n_chunks, n_out,
                       groups > 1 ? kReduceGroup : 1);
}

// WT[tap][ci][co] = W[co][tap][ci] (bf16) for the dgrad of a 32x32 layer
__global__ __launch_bounds__(256) void k_transpose_w(const uint16_t* __restrict__ Wt,
                                                     uint16_t* __restrict__ WT) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over co, t, ci
    if (i >= 32 * 9 * 32) return;
    const int co = i / 288, t = (i / 32) % 9, ci = i % 32;
    WT[((size_t)t * 32 + ci) * 32 + co] = Wt[i];
}

// Adam with bias correction on fp32 master weights; refreshes the bf16 copy
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, const float* __restrict__ grad,
                                              float* __restrict__ m, float* __restrict__ v,
                                              uint16_t* __restrict__ wbf, int n, float lr, float b1,
                                              float b2, float omb1, float omb2, float eps, float bc1,
                                              float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = b1 * m[i] + omb1 * g;  // omb = 1 - b, rounded once from the exact value
    const float vi = b2 * v[i] + omb2 * g * g;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    theta[i] = th;
    wbf[i] = f2bf(th);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ a, uint16_t* __restrict__ b,
                                                 int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = f2bf(a[i]);
}

// occluded fraction of every 16x16 tile (edge tiles partial): M uint8 [n][H][W]
__global__ __launch_bounds__(256) void k_tile_targets(const uint8_t* __restrict__ M, int n, int H,
                                                      int W, float* __restrict__ T) {
    const int Ht = (H + 15) / 16, Wt = (W + 15) / 16;
    const long total = (long)n * Ht * Wt;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long)gridDim.x * blockDim.x) {
        const int k = (int)(i / ((long)Ht * Wt));
        const int rem = (int)(i % ((long)Ht * Wt));
        const int ty = rem / Wt, tx = rem % Wt;
        const int y1 = min(H, ty * 16 + 16), x1 = min(W, tx * 16 + 16);
        int cnt = 0;
        for (int y = ty * 16; y < y1; ++y)
            for (int x = tx * 16; x < x1; ++x) cnt += M[((size_t)k * H + y) * W + x] != 0;
        T[i] = (float)cnt / (float)((y1 - ty * 16) * (x1 - tx * 16));
    }
}

inline int blocks_for(long n, int per, int cap) {
    long g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t cnn_pack(hipStream_t st, const float* D, int H, int W, int n_views, const ViewTable& vt,
                    const int* Ls, uint16_t* X) {
    PackViews pv{};
    for (int v = 0; v < n_views; ++v) {
        pv.c[v] = vt.c[v];
        pv.s[v] = vt.s[v];
        pv.r[v] = vt.r[v];
        pv.inv_L[v] = 1.0f / (float)Ls[v];
    }
    hipLaunchKernelGGL(k_pack, dim3(blocks_for((long)H * W, 256, 16384)), dim3(256), 0, st, D, H, W,
                       n_views, pv, X);
    return hipGetLastError();
}

hipError_t cnn_conv_fwd(hipStream_t st, int cin, int stride, const uint16_t* X, const uint16_t* Wt,
                        const float* b, uint16_t* Y, int N, int H, int W, int Ho, int Wo, int n_cu) {
    // persistent: as many 4-wavefront blocks as stay resident, each wavefront
    // walking 32-pixel tiles
    const long tiles = ((long)N * Ho * Wo + 31) / 32;
    const long resident = (long)n_cu * (cin == 8 ? 8 : 4);
    const dim3 grid((unsigned)std::max<long>(1, std::min<long>((tiles + 3) / 4, resident))), block(256);
    if (cin == 8 && stride == 2)
        hipLaunchKernelGGL((k_conv_fwd_p<8, 2>), grid, block, 0, st, X, Wt, b, Y, N, H, W, Ho, Wo);
    else if (cin == 32 && stride == 2)
        hipLaunchKernelGGL((k_conv_fwd_p<32, 2>), grid, block, 0, st, X, Wt, b, Y, N, H, W, Ho, Wo);
    else if (cin == 32 && stride == 1)
        hipLaunchKernelGGL((k_conv_fwd_p<32, 1>), grid, block, 0, st, X, Wt, b, Y, N, H, W, Ho, Wo);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t cnn_first_layer_fused(hipStream_t st, const float* D, int H, int W, int n_views,
                                 const ViewTable& vt, const int* Ls, uint4* G, const uint16_t* Wt,
                                 const float* b, uint16_t* Y, int Ho, int Wo, int n_cu) {
    PackViews pv{};
    for (int v = 0; v < n_views; ++v) {
        pv.c[v] = vt.c[v];
        pv.s[v] = vt.s[v];
        pv.r[v] = vt.r[v];
        pv.inv_L[v] = 1.0f / (float)Ls[v];
    }
    hipLaunchKernelGGL(k_pack_base, dim3(blocks_for((long)H * W, 256, 16384)), dim3(256), 0, st, D, H, W, G);
    const long tiles = ((long)Ho * Wo + 31) / 32;
    const dim3 grid((unsigned)std::max<long>(1, std::min<long>((tiles + 3) / 4, (long)n_cu * 8)));
    hipLaunchKernelGGL(k_conv0_fused, grid, dim3(256), 0, st, G, H, W, n_views, pv, Wt, b, Y, Ho, Wo);
    return hipGetLastError();
}

hipError_t cnn_first_layers_fused(hipStream_t st, const float* D, int H, int W, int n_views,
                                  const ViewTable& vt, const int* Ls, uint4* G, const uint16_t* W0,
                                  const float* b0, const uint16_t* W1, const float* b1, uint16_t* Y1,
                                  int H0, int W0n, int H1, int W1n, int n_cu) {
    PackViews pv{};
    for (int v = 0; v < n_views; ++v) {
        pv.c[v] = vt.c[v];
        pv.s[v] = vt.s[v];
        pv.r[v] = vt.r[v];
        pv.inv_L[v] = 1.0f / (float)Ls[v];
    }
    hipLaunchKernelGGL(k_pack_base, dim3(blocks_for((long)H * W, 256, 16384)), dim3(256), 0, st, D, H, W, G);
    constexpr int TY = 8;
    const long tiles = (long)((H1 + TY - 1) / TY) * ((W1n + 31) / 32);
    // one block per compute unit (its LDS holds the G window and the layer-0 tile)
    const dim3 grid((unsigned)std::max<long>(1, std::min<long>(tiles, (long)n_cu)));
    hipLaunchKernelGGL(k_conv01_fused<TY>, grid, dim3(64 * TY), 0, st, G, H, W, n_views, pv, W0, b0, W1, b1,
                       Y1, H0, W0n, H1, W1n);
    return hipGetLastError();
}

hipError_t cnn_conv_last(hipStream_t st, const uint16_t* X, const uint16_t* Wt, const float* b,
                         float* Z, int N, int H, int W) {
    hipLaunchKernelGGL(k_conv_last, dim3(blocks_for((long)N * H * W, 256, 65535)), dim3(256), 0, st,
                       X, Wt, b, Z, N, H, W);
    return hipGetLastError();
}

hipError_t cnn_bce(hipStream_t st, const float* Z, const float* T, float* dZ, double* partial, long n,
                   int n_blocks) {
    hipLaunchKernelGGL(k_bce, dim3(n_blocks), dim3(256), 0, st, Z, T, dZ, partial, n);
    return hipGetLastError();
}

hipError_t cnn_last_backward(hipStream_t st, const float* dZ, const uint16_t* X, const uint16_t* Wt,
                             uint16_t* dX, float* partial, float* gw_out, int N, int H, int W) {
    const long total = (long)N * H * W;
    const int chunk = kLastChunk;
    const int n_chunks = (int)((total + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_wgrad_last, dim3(n_chunks), dim3(320), 0, st, dZ, X, partial, N, H, W, chunk);
    reduce_chunks(st, partial, gw_out, n_chunks, 289);
    hipLaunchKernelGGL(k_dgrad_last, dim3(blocks_for(total * 32, 256, 65535)), dim3(256), 0, st, dZ, Wt,
                       dX, N, H, W);
    return hipGetLastError();
}

size_t cnn_last_partial_floats(long pixels) { return (size_t)((pixels + kLastChunk - 1) / kLastChunk) * 289; }

size_t cnn_wgrad_partial_floats(long pixels, int cin) {
    const int chunk = kWgradChunk;
    const long n_chunks = (pixels + chunk - 1) / chunk;
    return (size_t)n_chunks * 32 * 9 * cin + (size_t)n_chunks * 32;
}

// gw_out: dW [32][9*cin] then db [32]
hipError_t cnn_layer_backward(hipStream_t st, int cin, int stride, const uint16_t* dY,
                              const uint16_t* Y, const uint16_t* X, const uint16_t* Wt,
                              uint16_t* WT, uint16_t* dX, float* partial, float* gw_out, int N, int H,
                              int W, int Ho, int Wo) {
    const long total = (long)N * Ho * Wo;
    const int chunk = kWgradChunk;
    const int n_chunks = (int)((total + chunk - 1) / chunk);
    const int ncol = 9 * cin;
    const dim3 wg(n_chunks);
    if (cin == 8 && stride == 2)
        hipLaunchKernelGGL((k_conv_wgrad<8, 2>), wg, dim3(256), 0, st, dY, Y, X, partial, N, H, W, Ho, Wo, chunk);
    else if (cin == 32 && stride == 2)
        hipLaunchKernelGGL((k_conv_wgrad<32, 2>), wg, dim3(256), 0, st, dY, Y, X, partial, N, H, W, Ho, Wo, chunk);
    else if (cin == 32 && stride == 1)
        hipLaunchKernelGGL((k_conv_wgrad<32, 1>), wg, dim3(256), 0, st, dY, Y, X, partial, N, H, W, Ho, Wo, chunk);
    else
        return hipErrorInvalidValue;
    reduce_chunks(st, partial, gw_out, n_chunks, 32 * ncol + 32);  // dW and db in one pass
    if (dX) {  // input gradient (not needed for the first layer)
        if (cin != 32) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_transpose_w, dim3((32 * 9 * 32 + 255) / 256), dim3(256), 0, st, Wt, WT);
        const long waves = ((long)N * H * W + 31) / 32;
        const dim3 grid((unsigned)((waves + 3) / 4));
        if (stride == 2)
            hipLaunchKernelGGL(k_conv_dgrad<2>, grid, dim3(256), 0, st, dY, Y, WT, dX, N, H, W, Ho, Wo);
        else
            hipLaunchKernelGGL(k_conv_dgrad<1>, grid, dim3(256), 0, st, dY, Y, WT, dX, N, H, W, Ho, Wo);
    }
    return hipGetLastError();
}

hipError_t cnn_adam(hipStream_t st, float* theta, const float* grad, float* m, float* v, uint16_t* wbf,
                    int n, float lr, double b1, double b2, double eps, double bc1, double bc2) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, theta, grad, m, v, wbf, n, lr,
                       (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), (float)eps,
                       (float)bc1, (float)bc2);
    return hipGetLastError();
}

hipError_t cnn_to_bf16(hipStream_t st, const float* a, uint16_t* b, int n) {
    hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}

hipError_t cnn_tile_targets(hipStream_t st, const uint8_t* M, int n, int H, int W, float* T) {
    const long tiles = (long)n * ((H + 15) / 16) * ((W + 15) / 16);
    hipLaunchKernelGGL(k_tile_targets, dim3(blocks_for(tiles, 256, 65535)), dim3(256), 0, st, M, n, H, W, T);
    return hipGetLastError();
}

}  // namespace occl
