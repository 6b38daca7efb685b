// Per-voxel Adam update shared by the plain optimiser kernel and the fused
// gradient-smoothing + Adam kernel, so that both give bitwise the same field.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace ffdp {

// Step constants: the bias corrections are formed on the host in double.
struct AdamK {
    float b1, b2, eps, step_size, inv_sqrt_bc2;
};

inline AdamK adam_constants(float lr, float b1, float b2, float eps, int64_t step)
{
    AdamK k;
    k.b1 = b1; k.b2 = b2; k.eps = eps;
    const double bc1 = 1.0 - std::pow((double)b1, (double)step);
    const double bc2 = 1.0 - std::pow((double)b2, (double)step);
    k.step_size = (float)((double)lr / bc1);
    k.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
    return k;
}

// m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
// x <- x - lr/(1 - b1^t) m / (sqrt(v)/sqrt(1 - b2^t) + eps)
__device__ __forceinline__ void adam1(float& x, float g, float& m, float& v, const AdamK& k)
{
    m = fmaf(k.b1, m, (1.0f - k.b1) * g);
    v = fmaf(k.b2, v, (1.0f - k.b2) * g * g);
    x -= k.step_size * m / fmaf(sqrtf(v), k.inv_sqrt_bc2, k.eps);
}

// x, m, v [channels][D][H][W] <- Adam with the gradient smoothed by the
// Gaussian of radius R (taps w); g must not overlap x, m, v.
hipError_t smooth_adam_launch(float* x, const float* g, float* m, float* v, int D, int H, int W, int channels,
                              const float* w, int R, const AdamK& k, hipStream_t st);

}  // namespace ffdp
