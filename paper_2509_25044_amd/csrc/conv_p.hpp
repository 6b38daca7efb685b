// U-Net backward from a precomputed bf16 P = dL/dy act'(y) (host side of
// conv3d.hip; the entry points are ffdp_conv3d_act_grad,
// ffdp_conv3d_bwd_data_bf16 and ffdp_conv3d_bwd_weight_bf16).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace ffdp {

// P [n] bf16 = round-to-nearest-even(dy * act'(y)); y may be NULL (identity)
hipError_t act_grad_launch(const float* dy, const unsigned short* y, float slope, long long n, unsigned short* p,
                           hipStream_t st);
// conv_bwd_weight_launch with P (bf16, dL/dy's layout) instead of dy and y;
// the same workspace
hipError_t conv_bwd_weight_p_launch(const ConvGeom& g, const unsigned short* xa, const unsigned short* xb,
                                    const unsigned short* p, float* dw, float* db, float* part, hipStream_t st);
// conv_bwd_data_launch with P (bf16, dL/dy's layout) instead of dy and y
hipError_t conv_bwd_data_p_launch(const ConvGeom& g, const unsigned short* p, const unsigned short* wt, float* dx,
                                  int accumulate, hipStream_t st);

}  // namespace ffdp
