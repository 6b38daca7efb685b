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

}  // namespace ffdp
