// Host-side declarations shared between the C-ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ffdp {

// LNCC tile: 32 x 16 columns per block, 512 threads (8 waves of 64)
constexpr int LNCC_TX = 32;
constexpr int LNCC_TY = 16;
constexpr int LNCC_NT = 512;

struct LnccArgs {
    const float* F;
    const float* M;
    const float* u;       // [3][D][H][W] or null
    float* gu;            // [3][D][H][W] (bwd / ants modes)
    const float* grad_scale;
    double* partial;      // [nblocks]
    int D, H, W;
    int roi[6];           // z0, z1, y0, y1, x0, x1
    float eps;
    float neg_inv_nroi;   // -1 / N_roi
    int ntx, nty, zchunk, nblocks;
};

struct LnccLaunch {
    int ntx, nty, zchunk, nchunks, nblocks;
};

LnccLaunch lncc_plan(int D, int H, int W);
hipError_t lncc_launch(int mode, int win, int pad, const LnccArgs& a, float* loss, double nroi, hipStream_t st);

// MI
constexpr int MI_TX = 64;
constexpr int MI_TY = 4;
constexpr int MI_NT = MI_TX * MI_TY;

struct MiLaunch {
    int ntx, nty, zchunk, nchunks, nblocks;
};
MiLaunch mi_plan(int rz, int ry, int rx);

struct MiArgs {
    const float* F;
    const float* M;
    const float* u;
    int D, H, W;
    int roi[6];
    int bins;
    int ntx, nty, zchunk, nblocks;
};

hipError_t mi_fwd_launch(const MiArgs& a, int hard, int pad, unsigned long long* hist, float* state, float* loss,
                         double nroi, hipStream_t st);
hipError_t mi_bwd_launch(const MiArgs& a, int hard, int pad, const float* state, const float* grad_scale,
                         float* gu, double nroi, hipStream_t st);

// elementwise
hipError_t warp_launch(const float* M, const float* u, int D, int H, int W, int pad, float* out, hipStream_t st);
hipError_t resample_launch(const float* src, int sD, int sH, int sW, float* dst, int dD, int dH, int dW, int ch,
                           float scale, hipStream_t st);
hipError_t adam_launch(float* x, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t st);

// separable Gaussian smoothing: normalised taps w[0..2R], w[R] the centre
constexpr int SMOOTH_MAX_R = 6;
struct SmoothWeights {
    float w[2 * SMOOTH_MAX_R + 1];
};
hipError_t smooth_launch(const float* in, float* out, int D, int H, int W, int channels, const SmoothWeights& w,
                         int R, hipStream_t st);

// 3x3x3 convolutions of the warm-start network
struct ConvGeom {
    int N;
    int Di, Hi, Wi;  // convolution input (after upsampling)
    int Do, Ho, Wo;  // output
    int Ca, Cb;      // channels of the (optionally upsampled) part a and the skip part b
    int Cout;
    int stride;      // 1 or 2
    int ups;         // part a stored at half resolution, nearest x2
};
struct ConvWgradPlan {
    long long VC;          // output voxels per chunk
    int nchunks;
    long long part_floats;  // workspace floats
};
ConvWgradPlan conv_wgrad_plan(const ConvGeom& g);
hipError_t conv_fwd_launch(const ConvGeom& g, const unsigned short* xa, const unsigned short* xb,
                           const unsigned short* w, const float* bias, int act, float slope, unsigned short* ybf,
                           float* yf, hipStream_t st);
hipError_t conv_bwd_data_launch(const ConvGeom& g, const float* dy, const unsigned short* y, float slope,
                                const unsigned short* wt, float* dx, int accumulate, hipStream_t st);
hipError_t conv_bwd_weight_launch(const ConvGeom& g, const unsigned short* xa, const unsigned short* xb,
                                  const float* dy, const unsigned short* y, float slope, float* dw, float* db,
                                  float* part, hipStream_t st);
hipError_t cast_bf16_launch(const float* x, long long n, unsigned short* y, hipStream_t st);
hipError_t weight_prep_launch(const float* w, int Cout, int Cin, unsigned short* wbf, unsigned short* wt,
                              hipStream_t st);
hipError_t pack_pair_launch(const float* F, const float* M, long long nvox, unsigned short* x, hipStream_t st);
hipError_t split_grad_launch(const ConvGeom& g, const float* dxc, float* dxa, float* dxb, int acc_a, int acc_b,
                             hipStream_t st);
constexpr int MSE_BLOCKS = 1024;
hipError_t mse_launch(const float* pred, int Cp, const float* tgt, long long nvox_per, int N, float* dpred,
                      double* part, int nblocks, float* loss, hipStream_t st);
hipError_t unpack_disp_launch(const float* pred, int Cp, long long nvox_per, int N, float* u, hipStream_t st);

}  // namespace ffdp
