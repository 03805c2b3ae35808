// occl_cnn.h -- library-internal declarations of the learned tile proposal
// (kernels in k_cnn.hip, host side in occl_cnn.hip).
#pragma once

#include "occl_internal.h"

namespace occl {

// 6 layers of 3x3 convolutions; the logits come out on 16 x 16 pixel tiles.
constexpr int kCnnLayers = 6;
constexpr int kCnnTile = 16;
constexpr int kCnnInCh = 8;

size_t cnn_num_params();
// Spatial size after each layer: Hs[0] = H, Hs[l + 1] = ceil(Hs[l] / stride_l).
void cnn_dims(int H, int W, int* Hs, int* Ws);

hipError_t cnn_pack(hipStream_t st, const float* D, int H, int W, int n_views, const ViewTable& vt,
                    const int* Ls, uint16_t* X);
hipError_t cnn_conv_fwd(hipStream_t st, int cin, int stride, const uint16_t* X, const uint16_t* Wt,
                        const float* b, uint16_t* Y, int N, int H, int W, int Ho, int Wo, int n_cu);
// Layer 0 of every view straight from D (input packing fused; bit-identical
// to cnn_pack followed by cnn_conv_fwd).  G: workspace of H * W uint4.
hipError_t cnn_first_layer_fused(hipStream_t st, const float* D, int H, int W, int n_views,
                                 const ViewTable& vt, const int* Ls, uint4* G, const uint16_t* Wt,
                                 const float* b, uint16_t* Y, int Ho, int Wo, int n_cu);
// Layers 0 and 1 of every view straight from D, layer 0 never leaving LDS
// (bit-identical to cnn_pack, then cnn_conv_fwd twice).
hipError_t cnn_first_layers_fused(hipStream_t st, const float* D, int H, int W, int n_views,
                                  const ViewTable& vt, const int* Ls, uint4* G, const uint16_t* W0,
                                  const float* b0, const uint16_t* W1, const float* b1, uint16_t* Y1,
                                  int H0, int W0n, int H1, int W1n, int n_cu);
hipError_t cnn_conv_last(hipStream_t st, const uint16_t* X, const uint16_t* Wt, const float* b,
                         float* Z, int N, int H, int W);
hipError_t cnn_bce(hipStream_t st, const float* Z, const float* T, float* dZ, double* partial, long n,
                   int n_blocks);
hipError_t cnn_last_backward(hipStream_t st, const float* dZ, const uint16_t* X, const uint16_t* Wt,
                             uint16_t* dX, float* partial, float* gw_out, int N, int H, int W);
size_t cnn_wgrad_partial_floats(long pixels, int cin);
size_t cnn_last_partial_floats(long pixels);  // partials of cnn_last_backward over `pixels` logits
hipError_t cnn_layer_backward(hipStream_t st, int cin, int stride, const uint16_t* dY,
                              const uint16_t* Y, const uint16_t* X, const uint16_t* Wt,
                              uint16_t* WT, uint16_t* dX, float* partial, float* gw_out, int N, int H,
                              int W, int Ho, int Wo);
hipError_t cnn_adam(hipStream_t st, float* theta, const float* grad, float* m, float* v, uint16_t* wbf,
                    int n, float lr, double b1, double b2, double eps, double bc1, double bc2);
hipError_t cnn_to_bf16(hipStream_t st, const float* a, uint16_t* b, int n);
hipError_t cnn_tile_targets(hipStream_t st, const uint8_t* M, int n, int H, int W, float* T);

}  // namespace occl
