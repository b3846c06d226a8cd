// Convolutional surrogate: BF16 tensors, MFMA implicit-GEMM 3x3 convolutions.
//
// Activations are NHWC BF16 (raw 16-bit words), weights [C_out][3][3][C_in]
// BF16 for the forward product and [C_in][3][3][C_out] BF16 for the input
// gradient; master weights, gradients, Adam moments and every accumulation are
// FP32.  Channel counts are multiples of 8, so 8 consecutive reduction indices
// are 8 channels of one pixel and one tap: one 16-byte load per MFMA operand
// fragment.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vlbm {
namespace nn {

// One conv layer.  (H, W) is the full-resolution input of the convolution; with
// `up` the primary input is stored at (H/2, W/2) and read through a nearest 2x
// upsampling; `cskip` channels of a skip tensor at (H, W) follow the primary
// channels.  Output (OH, OW) = (ceil(H/stride), ceil(W/stride)).
struct Conv {
  int N, H, W;
  int cin, cskip, up, stride;
  int cout, relu;
  int OH, OW;
  __host__ __device__ int ctot() const { return cin + cskip; }
  __host__ __device__ int64_t out_pixels() const { return (int64_t)N * OH * OW; }
  __host__ __device__ int64_t in_pixels() const { return (int64_t)N * H * W; }
};

// returns an error text, or nullptr when the layer is one the kernels support
const char* check(const Conv& c);

hipError_t conv_forward(const Conv& c, const uint16_t* x, const uint16_t* skip, const uint16_t* w,
                        const float* bias, uint16_t* y16, float* y32, hipStream_t st);
// gx (primary input, stored resolution) and gskip accumulate (+=); either may be null.
// With g16 (and gx), the contribution to gx is taken to be its last: g16 = bf16(gx (act > 0))
// with act_relu, bf16(gx) without, the ReLU gradient of the layer whose output is the
// primary input (act, g16 in gx's layout), as relu_grad would form it.  assign_gx /
// assign_gskip: store the product instead of adding it (the tensor's first contribution).
hipError_t conv_backward_data(const Conv& c, const uint16_t* gy, const uint16_t* wt, float* gx, float* gskip,
                              hipStream_t st, const uint16_t* act = nullptr, int act_relu = 0,
                              uint16_t* g16 = nullptr, int assign_gx = 0, int assign_gskip = 0);
// gw [C_out][9][C_in + C_skip] and gb [C_out] accumulate (+=), or are stored with assign.  With a device
// workspace of at least conv_backward_weight_workspace(c) floats the partial
// sums are added in a fixed order (bit-reproducible); without one, with FP32
// atomics.
hipError_t conv_backward_weight(const Conv& c, const uint16_t* x, const uint16_t* skip, const uint16_t* gy,
                                float* gw, float* gb, hipStream_t st, float* work = nullptr,
                                int64_t work_floats = 0, int assign = 0);
int64_t conv_backward_weight_workspace(const Conv& c);
hipError_t pack_weights(const Conv& c, const float* w, uint16_t* w16, uint16_t* wt16, hipStream_t st);
// pack_weights for nlayers <= kMaxPackLayers layers in one launch; layer l's
// weights start at w_off[l] in params, w16 and wt16
constexpr int kMaxPackLayers = 32;
hipError_t pack_weights_all(int nlayers, const Conv* convs, const int64_t* w_off, const float* params, uint16_t* w16,
                            uint16_t* wt16, hipStream_t st);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st);
hipError_t fill(float* p, int64_t n, float v, hipStream_t st);
// out16 = bf16(g * (act > 0)) with relu, bf16(g) without
hipError_t relu_grad(const float* g, const uint16_t* act, uint16_t* out16, int64_t n, int relu, hipStream_t st);
// [pixels][cin] FP32 -> [pixels][cpad] BF16, zero-filled channels
hipError_t pack_input(const float* x, uint16_t* x16, int64_t pixels, int cin, int cpad, hipStream_t st);
// y[pixels][cout] = out[pixels][cpad] for the first cout channels
hipError_t unpack_output(const float* out, float* y, int64_t pixels, int cpad, int cout, hipStream_t st);
// loss = sum (out - t)^2 / count over the first ct channels (in a fixed order; part: device
// workspace of kMseBlocks doubles); gout = 2 (out - t) / count there, 0 elsewhere
constexpr int kMseBlocks = 4096;
hipError_t mse(const float* out, const float* t, float* gout, double* loss, int64_t pixels, int cpad, int ct,
               double* part, hipStream_t st);

}  // namespace nn
}  // namespace vlbm
