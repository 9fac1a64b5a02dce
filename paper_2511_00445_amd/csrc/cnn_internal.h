// Internal interface of the surrogate network's kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tcnn {

using bf16 = uint16_t;  // raw bfloat16 storage

constexpr int kChannels = 7, kHidden = 48, kLayers = 6;
constexpr int kPadIO = 16;  // the 7 state channels padded to one MFMA k-block
constexpr int kTile = 16;   // output tile: 16 x 16 sites

// Epilogue of the convolution kernel.
enum ConvMode {
  kSilu = 0,    // z = acc + b (stored fp32 when given), a = bf16(silu(z))
  kLinear = 1,  // y = acc + b (fp32)
  kBackward = 2 // g = bf16(acc * silu'(z_below))
};

// One periodic 3x3 convolution over B images of H x W sites (H, W multiples of 16).
// in: [B][H][W][ci] bf16; w: [co][9][ci] bf16 (tap = 3 dy + dx); bias: [co] fp32.
hipError_t launch_conv(int ci, int co, ConvMode mode, const bf16* in, const bf16* w, const float* bias,
                       const float* z_below, bf16* out_bf, float* out_f, int B, int H, int W, hipStream_t st);

// Weight and bias gradients of one layer: block partials, then a fixed-order sum
// into the natural layout gW[co][ci][3][3] and gb[co] of the real channels.
int dw_blocks(int B, int H, int W);
hipError_t launch_weight_grad(int ci, int co, int ci_real, int co_real, const bf16* g, const bf16* a,
                              float* partial, float* partial_b, float* gW, float* gb, int B, int H, int W,
                              hipStream_t st);

// State [n][7][H][W] fp32 (sample idx[b] of a stacked array) -> bf16 [B][H][W][16] / scale.
hipError_t launch_pack(const float* x, int64_t sample_stride, const int* idx, const float* inv_scale,
                       bf16* a0, int B, int H, int W, hipStream_t st);
// Loss terms: d = y - (target - x) / s; g = bf16(2 d / count); per-block sums of d^2.
int loss_blocks(int B, int H, int W);
hipError_t launch_loss(const float* y, const float* x, const float* target, int64_t sample_stride,
                       const int* idx, const float* inv_scale, bf16* g, double* partial, double* loss,
                       int B, int H, int W, hipStream_t st);
// Prediction x + s * y into out [B][7][H][W].
hipError_t launch_unpack(const float* y, const float* x, const float* scale, float* out, int B, int H, int W,
                         hipStream_t st);
// Adam on the fp32 parameter vector; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int64_t n, float lr, double beta1,
                       double beta2, float eps, float c1, float c2, hipStream_t st);
// bf16 forward ([co][9][ci]) and backward-data ([ci][9][co], taps reversed)
// copies of one layer's weights, padded with zeros, and the padded fp32 bias.
hipError_t launch_pack_weights(const float* W, const float* b, int ci_real, int co_real, int ci, int co,
                               bf16* wf, bf16* wb, float* bias, hipStream_t st);
// Per-channel sums of (a - b)^2 and b^2 over [B][7][H][W] (fp64, fixed order).
hipError_t launch_compare(const float* a, const float* b, int64_t plane, int B, double* partial,
                          double* out, hipStream_t st);
int compare_blocks(int64_t plane, int B);

}  // namespace tcnn
