// Separable 3D Gaussian smoothing of multi-channel fields, one pass over HBM
// (the gradient and warp smoothing of the paper's registration loop,
// sigma_grad = 1 and sigma_warp = 0.5 voxels).
//
//   out[c](z,y,x) = sum_{a,b,d} g(a) g(b) g(d) in[c](clamp(z+a), clamp(y+b), clamp(x+d))
//   g(t) = exp(-t^2 / (2 sigma^2)) / sum_{|s|<=R} exp(-s^2 / (2 sigma^2)),  |t| <= R
//
// with edge replication outside the array.  A block owns a 64 x 8 column
// tile of one channel and streams z: each slice (plus an R halo in x and y)
// is staged in LDS, filtered in x then y, and the last 2R+1 y-filtered
// slices of the thread's voxels stay in registers for the z filter.  HBM
// traffic is one read and one write per element plus the z halo of each
// chunk (2R slices per chunk of at least 32).
#include "device.hpp"
#include "internal.hpp"

namespace ffdp {

constexpr int SM_TX = 64, SM_TY = 16, SM_NT = 256;

template <int R>
__global__ void __launch_bounds__(SM_NT) smooth_kernel(const float* __restrict__ in, float* __restrict__ out, int D,
                                                       int H, int W, SmoothWeights wts, int zchunk, int nty)
{
    constexpr int X2 = SM_TX + 2 * R, Y2 = SM_TY + 2 * R, K = 2 * R + 1;
    constexpr int P = SM_TX * SM_TY / SM_NT;  // voxels per thread (4)
    __shared__ float s0[Y2 * X2];
    __shared__ float s1[Y2 * SM_TX];
    const int c = blockIdx.z;
    const int tx = blockIdx.x, ty = blockIdx.y % nty, ch = blockIdx.y / nty;
    const int gx0 = tx * SM_TX, gy0 = ty * SM_TY;
    const int z0 = ch * zchunk, z1 = min(D, z0 + zchunk);
    const size_t N = (size_t)D * H * W;
    const float* src = in + (size_t)c * N;
    float* dst = out + (size_t)c * N;
    const int tid = threadIdx.x;
    float g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) g[k] = wts.w[k];
    float ring[P][K];
    const int nsteps = (z1 - z0) + 2 * R;
    for (int base = 0; base < nsteps; base += K) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int s = base + j;
            if (s >= nsteps) break;
            const int zi = min(max(z0 - R + s, 0), D - 1);
            // stage the slice with an R halo (edge replication)
            for (int p = tid; p < Y2 * X2; p += SM_NT) {
                const int ly = p / X2, lx = p - ly * X2;
                const int gx = min(max(gx0 - R + lx, 0), W - 1), gy = min(max(gy0 - R + ly, 0), H - 1);
                s0[p] = src[(size_t)zi * H * W + (size_t)gy * W + gx];
            }
            __syncthreads();
            for (int p = tid; p < Y2 * SM_TX; p += SM_NT) {
                const int ly = p / SM_TX, lx = p - ly * SM_TX;
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc = fmaf(g[k], s0[ly * X2 + lx + k], acc);
                s1[p] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int p = tid + q * SM_NT;
                const int ly = p / SM_TX, lx = p - ly * SM_TX;
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc = fmaf(g[k], s1[(ly + k) * SM_TX + lx], acc);
                ring[q][j] = acc;
                const int zo = z0 + s - 2 * R;  // output slice, valid once the ring is full
                const int gx = gx0 + lx, gy = gy0 + ly;
                if (s >= 2 * R && gx < W && gy < H) {
                    float o = 0.f;
                    // ring slot of slice zo - R + k is (j + 1 + k) % K
#pragma unroll
                    for (int k = 0; k < K; ++k) o = fmaf(g[k], ring[q][(j + 1 + k) % K], o);
                    dst[(size_t)zo * H * W + (size_t)gy * W + gx] = o;
                }
            }
            __syncthreads();  // s0/s1 reused by the next slice
        }
    }
}

hipError_t smooth_launch(const float* in, float* out, int D, int H, int W, int channels, const SmoothWeights& w,
                         int R, hipStream_t st)
{
    const int ntx = (W + SM_TX - 1) / SM_TX, nty = (H + SM_TY - 1) / SM_TY;
    const int tiles = ntx * nty;
    int chunks = (2048 + tiles * channels - 1) / (tiles * channels);
    const int maxchunks = (D + 31) / 32;
    if (chunks > maxchunks) chunks = maxchunks;
    if (chunks < 1) chunks = 1;
    const int zchunk = (D + chunks - 1) / chunks;
    chunks = (D + zchunk - 1) / zchunk;
    dim3 grid(ntx, nty * chunks, channels), block(SM_NT);
    switch (R) {
        case 1: hipLaunchKernelGGL(smooth_kernel<1>, grid, block, 0, st, in, out, D, H, W, w, zchunk, nty); break;
        case 2: hipLaunchKernelGGL(smooth_kernel<2>, grid, block, 0, st, in, out, D, H, W, w, zchunk, nty); break;
        case 3: hipLaunchKernelGGL(smooth_kernel<3>, grid, block, 0, st, in, out, D, H, W, w, zchunk, nty); break;
        case 4: hipLaunchKernelGGL(smooth_kernel<4>, grid, block, 0, st, in, out, D, H, W, w, zchunk, nty); break;
        case 5: hipLaunchKernelGGL(smooth_kernel<5>, grid, block, 0, st, in, out, D, H, W, w, zchunk, nty); break;
        case 6: hipLaunchKernelGGL(smooth_kernel<6>, grid, block, 0, st, in, out, D, H, W, w, zchunk, nty); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ffdp
