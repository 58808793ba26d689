// Multi-channel stencil layer (3 x 3, NHWC bf16 activations).
#pragma once

#include "common.h"

namespace rise {

struct ConvArgs {
  uint16_t* out;
  const uint16_t* in;
  const float* w;  // Cout x Cin x 3 x 3
  int B, Cin, Cout, H, W;
  int zero_pad;
};
struct ConvBwdArgs {
  uint16_t* din;  // may be null
  float* dw;      // may be null
  const uint16_t* dout;
  const uint16_t* in;
  const float* w;
  int B, Cin, Cout, H, W;
  int zero_pad;
};
bool conv_supported(int Cin, int Cout, int kh, int kw, bool backward);
size_t conv_forward_workspace(int Cin, int Cout);
size_t conv_backward_workspace(int B, int Cin, int Cout, int H, int W);
rise_status launch_conv2d(const ConvArgs& a, void* ws, hipStream_t s);
rise_status launch_conv2d_backward(const ConvBwdArgs& a, void* ws, hipStream_t s);

}  // namespace rise
