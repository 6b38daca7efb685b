// Host-side declarations shared between the C-ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ffdp {

// LNCC launch arguments.  Tile sizes are chosen per window and mode by
// lncc_plan (32 x 32 columns with 1024 threads, or 32 x 16 with 512).
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
    int zspan;            // slices addressable with 32-bit byte offsets from one slice (windowed addressing)
};

enum { LNCC_ADDR32 = 0, LNCC_ADDRWIN = 1, LNCC_ADDR64 = 2 };

struct LnccLaunch {
    int tx, ty, nt;       // tile columns and threads per block
    int ntx, nty, zchunk, nchunks, nblocks;
    int addr, zspan;      // addressing mode and window (slices)
};

// mode: 0 forward, 1 adjoint, 2 ANTs adjoint
LnccLaunch lncc_plan(int D, int H, int W, int win, int mode);
// workspace blocks: the largest plan over the modes of one window
int lncc_max_blocks(int D, int H, int W, int win);
hipError_t lncc_launch(int mode, int win, int pad, const LnccLaunch& L, const LnccArgs& a, float* loss, double nroi,
                       hipStream_t st);

// Composite sampler, affine part: the sample point of voxel X = (x, y, z) is
// X + d with d = Am X + t + S u(X) and Am = A - I formed on the host in
// double, so that the identity transform gives d = u exactly.
struct Affine {
    float Am[9];  // row-major, acting on (x, y, z)
    float t[3];
    float S[9];   // row-major, acting on (u_x, u_y, u_z)
};

__device__ __forceinline__ void affine_disp(const Affine& f, int x, int y, int z, float ux, float uy, float uz,
                                            float& dx, float& dy, float& dz)
{
    const float X = (float)x, Y = (float)y, Z = (float)z;
    dx = fmaf(f.Am[0], X, fmaf(f.Am[1], Y, fmaf(f.Am[2], Z, f.t[0]))) + fmaf(f.S[0], ux, fmaf(f.S[1], uy, f.S[2] * uz));
    dy = fmaf(f.Am[3], X, fmaf(f.Am[4], Y, fmaf(f.Am[5], Z, f.t[1]))) + fmaf(f.S[3], ux, fmaf(f.S[4], uy, f.S[5] * uz));
    dz = fmaf(f.Am[6], X, fmaf(f.Am[7], Y, fmaf(f.Am[8], Z, f.t[2]))) + fmaf(f.S[6], ux, fmaf(f.S[7], uy, f.S[8] * uz));
}

// Adjoint of the affine part for one voxel: with g = dL/dMw dMw/dp, adds
// g X^T to acc[0..8] (row-major dL/dA) and g to acc[9..11] (dL/dt), and
// returns S^T g (dL/du) in gx, gy, gz.
__device__ __forceinline__ void affine_adjoint(const Affine& f, int x, int y, int z, float g0, float g1, float g2,
                                               double acc[12], float& gx, float& gy, float& gz)
{
    const double X = x, Y = y, Z = z;
    const double G[3] = {g0, g1, g2};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        acc[3 * i + 0] = fma(G[i], X, acc[3 * i + 0]);
        acc[3 * i + 1] = fma(G[i], Y, acc[3 * i + 1]);
        acc[3 * i + 2] = fma(G[i], Z, acc[3 * i + 2]);
        acc[9 + i] += G[i];
    }
    gx = fmaf(f.S[0], g0, fmaf(f.S[3], g1, f.S[6] * g2));
    gy = fmaf(f.S[1], g0, fmaf(f.S[4], g1, f.S[7] * g2));
    gz = fmaf(f.S[2], g0, fmaf(f.S[5], g1, f.S[8] * g2));
}

// dL/dA, dL/dt: fixed-order sum of per-block partials part[12 * b + q] -> out[12]
hipError_t affine_reduce_launch(const double* part, int nblocks, double* out, hipStream_t st);

// MI
constexpr int MI_MAX_BINS = 256;
constexpr int MI_LDS_TABLE_BINS = 128;  // log tables up to 128^2 floats (64 KB) are staged in LDS
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
    int ncopy;       // LDS histogram copies, a power of two (set by mi_fwd_launch)
    int affine;      // 1: composite sampler with aff
    Affine aff;
    double* apart;   // [nblocks][12] partial dL/dA, dL/dt (affine adjoint)
};

hipError_t mi_fwd_launch(const MiArgs& a, int hard, int pad, unsigned long long* hist, float* state, float* loss,
                         double nroi, hipStream_t st);
hipError_t mi_bwd_launch(const MiArgs& a, int hard, int pad, const float* state, const float* grad_scale,
                         float* gu, double nroi, hipStream_t st);

// checked mode: flag = 0, then flag |= any non-finite value of p[0..n)
hipError_t finite_clear_launch(unsigned* flag, hipStream_t st);
hipError_t finite_check_launch(const float* p, long long n, unsigned* flag, hipStream_t st);

// elementwise
hipError_t warp_launch(const float* M, const float* u, int D, int H, int W, int pad, float* out, hipStream_t st);
hipError_t warp_affine_launch(const float* M, const float* u, int D, int H, int W, const Affine& f, int pad,
                              float* out, hipStream_t st);
// adjoint of the composite warp for an upstream gradient gout; gu nullable;
// part: [nblocks][12] with nblocks = mi_plan(D, H, W).nblocks
hipError_t warp_affine_bwd_launch(const float* M, const float* u, int D, int H, int W, const Affine& f, int pad,
                                  const float* gout, float* gu, double* part, double* gAt, hipStream_t st);
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
    long long VC;          // output voxels per chunk (bias partials; the voxel-chunk kernels)
    int nchunks;
    long long part_floats;  // workspace floats
    int rows;              // 1: the row-segment kernel (stride 1, Cout <= 64)
    long long VS;          // row segments of 32 output voxels per chunk (row-segment kernel)
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
