// Separable 3D Gaussian smoothing of multi-channel fields, one pass over HBM
// (the gradient and warp smoothing of the paper's registration loop,
// sigma_grad = 1 and sigma_warp = 0.5 voxels).
//
//   out[c](z,y,x) = sum_{a,b,d} g(a) g(b) g(d) in[c](clamp(z+a), clamp(y+b), clamp(x+d))
//   g(t) = exp(-t^2 / (2 sigma^2)) / sum_{|s|<=R} exp(-s^2 / (2 sigma^2)),  |t| <= R
//
// with edge replication outside the array.  A block owns a 64 x 16 column
// tile of one channel and streams z.  Per slice:
//  1. the slice plus an R halo in x and y, loaded into registers during the
//     previous slice, is written to LDS;
//  2. the loads of the next slice are issued (they complete while this slice
//     is filtered, so HBM latency is hidden behind the LDS passes);
//  3. x filter: a thread forms 4 consecutive outputs of a row from one run of
//     aligned float4 LDS reads;
//  4. y filter: a thread forms 4 consecutive rows of one column from 4 + 2R
//     LDS reads, and the last 2R+1 y-filtered slices of its 4 voxels stay in
//     registers for the z filter, whose output is written to HBM.
// Two barriers per slice (the write of step 1 and the x outputs of step 3).
// HBM traffic is one read and one write per element plus the z halo of each
// chunk (2R slices per chunk of at least 32).
//
// The ADAM variant applies the optimiser step to (x, m, v) with the smoothed
// value as the gradient where the plain kernel would store it: the smoothed
// gradient of the registration loop never reaches HBM (8 bytes per element,
// 24 per voxel of a displacement field, saved against smoothing then
// stepping), with bitwise the same result.
#include "adam.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace ffdp {

constexpr int SM_TX = 64, SM_TY = 16, SM_NT = 256;

template <int R>
struct SmoothTile {
    static constexpr int K = 2 * R + 1;
    static constexpr int X2 = SM_TX + 2 * R, Y2 = SM_TY + 2 * R;
    static constexpr int NF4 = (K + 3 + 3) / 4;             // float4 reads per 4-output x run
    static constexpr int X2p = (SM_TX + 4 * NF4 > X2 ? SM_TX + 4 * NF4 : X2 + 3) & ~3;  // s0 row pitch
    static constexpr int NS0 = Y2 * X2;                     // staged elements per slice
    static constexpr int PL = (NS0 + SM_NT - 1) / SM_NT;    // staged elements per thread
    static constexpr int RX = Y2 * (SM_TX / 4);             // x runs per slice
    static_assert(SM_TX * SM_TY == 4 * SM_NT, "4 voxels per thread");
    static_assert(X2p >= SM_TX - 4 + 4 * NF4, "x runs stay inside the row");
};

template <int R, bool ADAM>
__global__ void __launch_bounds__(SM_NT) smooth_kernel(const float* __restrict__ in, float* __restrict__ out, int D,
                                                       int H, int W, SmoothWeights wts, int zchunk, int nty,
                                                       float* __restrict__ am, float* __restrict__ av, AdamK ak)
{
    using T = SmoothTile<R>;
    constexpr int K = T::K, X2 = T::X2, X2p = T::X2p, PL = T::PL;
    __shared__ __attribute__((aligned(16))) float s0[T::Y2 * X2p];
    __shared__ __attribute__((aligned(16))) float s1[T::Y2 * SM_TX];
    const int c = blockIdx.z;
    const int tx = blockIdx.x, ty = blockIdx.y % nty, ch = blockIdx.y / nty;
    const int gx0 = tx * SM_TX, gy0 = ty * SM_TY;
    const int z0 = ch * zchunk, z1 = min(D, z0 + zchunk);
    const size_t N = (size_t)D * H * W;
    const size_t HW = (size_t)H * W;
    const float* src = in + (size_t)c * N;
    float* dst = out + (size_t)c * N;
    const int tid = threadIdx.x;
    float g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) g[k] = wts.w[k];

    // staged elements of this thread: in-slice offsets (clamped: edge
    // replication, every load in bounds) and LDS slots
    unsigned soff[PL];
    int slot[PL];
#pragma unroll
    for (int i = 0; i < PL; ++i) {
        const int p = tid + i * SM_NT;
        const int ly = p / X2, lx = p - ly * X2;
        const int gx = min(max(gx0 - R + lx, 0), W - 1), gy = min(max(gy0 - R + ly, 0), H - 1);
        soff[i] = (unsigned)(gy * W + gx);
        slot[i] = p < T::NS0 ? ly * X2p + lx : -1;
    }
    float pre[PL];
    auto load_slice = [&](int s) {
        const float* sl = src + (size_t)min(max(z0 - R + s, 0), D - 1) * HW;
#pragma unroll
        for (int i = 0; i < PL; ++i) pre[i] = sl[soff[i]];
    };

    // y/z stage: column yx, rows 4*yg .. 4*yg+3 of the tile
    const int yx = tid % SM_TX, yg = tid / SM_TX;
    const int gx = gx0 + yx;
    float ring[4][K];
    const int nsteps = (z1 - z0) + 2 * R;
    load_slice(0);
    for (int base = 0; base < nsteps; base += K) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int s = base + j;
            if (s >= nsteps) break;
#pragma unroll
            for (int i = 0; i < PL; ++i)
                if (slot[i] >= 0) s0[slot[i]] = pre[i];
            __syncthreads();
            if (s + 1 < nsteps) load_slice(s + 1);
            // x filter: 4 outputs per run from aligned float4 reads
            for (int q = tid; q < T::RX; q += SM_NT) {
                const int ly = q / (SM_TX / 4), lx0 = 4 * (q - ly * (SM_TX / 4));
                float v[4 * T::NF4];
                const float4* row = reinterpret_cast<const float4*>(s0 + ly * X2p + lx0);
#pragma unroll
                for (int n = 0; n < T::NF4; ++n) {
                    const float4 t = row[n];
                    v[4 * n] = t.x; v[4 * n + 1] = t.y; v[4 * n + 2] = t.z; v[4 * n + 3] = t.w;
                }
                float4 o;
                float* op = reinterpret_cast<float*>(&o);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k < K; ++k) acc = fmaf(g[k], v[e + k], acc);
                    op[e] = acc;
                }
                *reinterpret_cast<float4*>(s1 + ly * SM_TX + lx0) = o;
            }
            __syncthreads();
            // y filter of 4 consecutive rows, then the z ring
            float col[4 + 2 * R];
#pragma unroll
            for (int n = 0; n < 4 + 2 * R; ++n) col[n] = s1[(4 * yg + n) * SM_TX + yx];
            const int zo = z0 + s - 2 * R;  // output slice, valid once the ring is full
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc = fmaf(g[k], col[e + k], acc);
                ring[e][j] = acc;
                const int gy = gy0 + 4 * yg + e;
                if (s >= 2 * R && gx < W && gy < H) {
                    float o = 0.f;
                    // ring slot of slice zo - R + k is (j + 1 + k) % K
#pragma unroll
                    for (int k = 0; k < K; ++k) o = fmaf(g[k], ring[e][(j + 1 + k) % K], o);
                    const size_t idx = (size_t)zo * HW + (size_t)gy * W + gx;
                    // every output byte is touched once: non-temporal accesses
                    if (ADAM) {  // out is x; m, v at the same offsets
                        const size_t ci = (size_t)c * N + idx;
                        float xx = __builtin_nontemporal_load(dst + idx);
                        float mm = __builtin_nontemporal_load(am + ci), vv = __builtin_nontemporal_load(av + ci);
                        adam1(xx, o, mm, vv, ak);
                        __builtin_nontemporal_store(xx, dst + idx);
                        __builtin_nontemporal_store(mm, am + ci);
                        __builtin_nontemporal_store(vv, av + ci);
                    } else {
                        __builtin_nontemporal_store(o, dst + idx);
                    }
                }
            }
        }
    }
}

template <bool ADAM>
static hipError_t smooth_dispatch(const float* in, float* out, int D, int H, int W, int channels,
                                  const SmoothWeights& w, int R, float* am, float* av, const AdamK& ak, hipStream_t st)
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
#define FFDP_SMOOTH_CASE(RR)                                                                                    \
    case RR:                                                                                                     \
        hipLaunchKernelGGL((smooth_kernel<RR, ADAM>), grid, block, 0, st, in, out, D, H, W, w, zchunk, nty, am, av, \
                           ak);                                                                                  \
        break;
    switch (R) {
        FFDP_SMOOTH_CASE(1)
        FFDP_SMOOTH_CASE(2)
        FFDP_SMOOTH_CASE(3)
        FFDP_SMOOTH_CASE(4)
        FFDP_SMOOTH_CASE(5)
        FFDP_SMOOTH_CASE(6)
        default: return hipErrorInvalidValue;
    }
#undef FFDP_SMOOTH_CASE
    return hipGetLastError();
}

hipError_t smooth_launch(const float* in, float* out, int D, int H, int W, int channels, const SmoothWeights& w,
                         int R, hipStream_t st)
{
    return smooth_dispatch<false>(in, out, D, H, W, channels, w, R, nullptr, nullptr, AdamK{}, st);
}

hipError_t smooth_adam_launch(float* x, const float* g, float* m, float* v, int D, int H, int W, int channels,
                              const float* taps, int R, const AdamK& k, hipStream_t st)
{
    SmoothWeights w{};
    for (int t = 0; t <= 2 * R; ++t) w.w[t] = taps[t];
    return smooth_dispatch<true>(g, x, D, H, W, channels, w, R, m, v, k, st);
}

}  // namespace ffdp
