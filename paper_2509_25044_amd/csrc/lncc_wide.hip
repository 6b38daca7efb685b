// Warp + LNCC forward and adjoint for wide windows (w = 11, 13, 15) on gfx950.
//
// The quantities are those of the fused kernel (App. "Definition of LNCC
// loss", eq. lncc-loss and lncc-a/b/c; the adjoint of eq. finalccgradM redone
// for the warped image with eps kept):
//   box sums of F, Mw, F^2, Mw^2, F Mw over the w^3 window, zero padding;
//   A, B, C, n_i = A^2 / (B C + eps), loss = 1 - mean_{ROI} n_i;
//   a_i = 2 g_i A_i / D_i, c_i = a_i A_i B_i / D_i, e_i = c_i mu_M,i - a_i mu_F,i
//   dL/dMw_k = (F_k (w*a)_k - Mw_k (w*c)_k + (w*e)_k) / w^3,  dL/du = dL/dMw dMw/dp.
// The fused kernel keeps the last w slices of every sampled column in
// registers and samples a 2r halo around each tile; past w = 9 those rings
// exceed a wave's registers, so here the window sums go through an FP64
// workspace in HBM in four passes:
//   1. wide_xy_kernel<5, SAMPLE>: per slice and 32 x 32 tile, sample F and Mw
//      on the tile plus an r halo into LDS, box the five products (formed in
//      FP64, exactly) along x then y, and write the xy sums S[5][N];
//   2. wide_z_kernel<MODE>: per (x, y) column, a running FP64 z-window sum of
//      S gives the box sums; the statistics, the loss term (FP64 block
//      partials, fixed-order finalize) and a, c, e (zero outside the ROI)
//      -> E[3][N] in fp32.  The ANTs mode (App. "ANTs gradient
//      approximation") writes its gradient here and stops;
//   3. wide_xy_kernel<3, LOAD>: xy box of E (32 x 16 tiles, FP64 sums)
//      -> T[3][N] in fp32, stored over S;
//   4. wide_grad_kernel: running FP64 z-window sum of T, Mw and dMw/dp
//      resampled at the voxel, grad_u written over the whole array.
// FP64 for S makes the cancellation in B = mu_FF - mu_F^2 harmless without a
// shift; every running sum accumulates in FP64 registers, free of drift over
// thousands of slices.  a, c, e and their xy sums are stored in fp32 (the
// precision the fused kernel keeps them in), which halves their traffic.
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"
#include "wide.hpp"

namespace ffdp {

namespace {

enum { WMODE_FWD = 0, WMODE_BWD = 1, WMODE_ANTS = 2 };

constexpr int WTX = 32, WXT = 512;                  // slice tile width and threads of the xy passes
constexpr int WNT = 256;                             // threads of the z passes
constexpr int WTY_S = 32, WTY_L = 16;                // tile heights: sampling pass, a/c/e pass
constexpr int WSEG = 8;                              // x outputs per thread in the sliding x-window
constexpr int WMAXR = (LNCC_MAX_WINDOW - 1) / 2;
constexpr int WX2 = WTX + 2 * WMAXR;
constexpr int WCX = 64, WCY = 4;                    // columns of the z passes (WCX * WCY = WNT)
static_assert(WCX * WCY == WNT, "one column per thread");
static_assert(WTX / WSEG * (WTY_S + 2 * WMAXR) <= WXT && WTX / WSEG * (WTY_L + 2 * WMAXR) <= WXT,
              "one x-window run per thread");
static_assert(WTY_S % (WXT / WTX) == 0 && WTY_L % (WXT / WTX) == 0, "whole rows per thread in the y-window");

struct WideArgs {
    const float* F;
    const float* M;
    const float* u;
    float* gu;
    const float* grad_scale;
    double* S;        // [5][N] xy sums (FP64); later [3][N] xy sums of a, c, e (fp32) over it
    float* E;         // [3][N] a, c, e (fp32, as the fused kernel keeps them)
    double* partial;  // [nblocks of the z passes]
    int D, H, W;
    int roi[6];
    int r;
    double eps;
    double neg_inv_nroi;
    int ntx;          // slice tiles along x
    int ncx, ncy, zchunk;
};

// Border-mode sample whose two x corners of each (row, slice) come as one
// 8-byte load (W >= 2): a point clamped at the low x border takes the first
// of the pair with weight 0, at the high border the second with weight 1
// (equal to it up to one rounding), and its x derivative is zero.  Along y
// and z the corner indices are clamped, as in trilinear_clamped.
typedef float wide_f2a __attribute__((ext_vector_type(2), aligned(4)));
template <bool DERIV>
__device__ __forceinline__ Tri sample_pair(const float* __restrict__ M, int D, int H, int W, int x, int y, int z,
                                           float ux, float uy, float uz)
{
    const float fx = fminf(fmaxf(floorf(ux), -268435456.0f), 268435456.0f);
    const float fy = fminf(fmaxf(floorf(uy), -268435456.0f), 268435456.0f);
    const float fz = fminf(fmaxf(floorf(uz), -268435456.0f), 268435456.0f);
    const float ax = ux - fx, ay = uy - fy, az = uz - fz;
    const int ix = x + (int)fx, iy = y + (int)fy, iz = z + (int)fz;
    const bool xlo = ix < 0, xhi = ix >= W - 1;
    const int xp = min(max(ix, 0), W - 2);
    const float axp = xlo ? 0.0f : (xhi ? 1.0f : ax);
    const int y0 = min(max(iy, 0), H - 1), y1 = min(max(iy + 1, 0), H - 1);
    const int z0 = min(max(iz, 0), D - 1), z1 = min(max(iz + 1, 0), D - 1);
    const int HW = H * W;  // D H W < 2^31: every index below fits an int
    const wide_f2a v00 = *reinterpret_cast<const wide_f2a*>(M + (z0 * HW + y0 * W + xp));
    const wide_f2a v01 = *reinterpret_cast<const wide_f2a*>(M + (z0 * HW + y1 * W + xp));
    const wide_f2a v10 = *reinterpret_cast<const wide_f2a*>(M + (z1 * HW + y0 * W + xp));
    const wide_f2a v11 = *reinterpret_cast<const wide_f2a*>(M + (z1 * HW + y1 * W + xp));
    const float e00 = v00.y - v00.x, e01 = v01.y - v01.x, e10 = v10.y - v10.x, e11 = v11.y - v11.x;
    const float c00 = fmaf(axp, e00, v00.x), c01 = fmaf(axp, e01, v01.x);
    const float c10 = fmaf(axp, e10, v10.x), c11 = fmaf(axp, e11, v11.x);
    const float f0 = c01 - c00, f1 = c11 - c10;
    const float c0 = fmaf(ay, f0, c00), c1 = fmaf(ay, f1, c10);
    Tri t;
    t.v = fmaf(az, c1 - c0, c0);
    if (DERIV) {
        const float gx0 = fmaf(ay, e01 - e00, e00), gx1 = fmaf(ay, e11 - e10, e10);
        t.dx = (xlo || xhi || (ix == 0 && ax == 0.0f)) ? 0.0f : fmaf(az, gx1 - gx0, gx0);
        t.dy = (iy == 0 && ay == 0.0f) ? 0.0f : fmaf(az, f1 - f0, f0);
        t.dz = (iz == 0 && az == 0.0f) ? 0.0f : (c1 - c0);
    } else {
        t.dx = t.dy = t.dz = 0.0f;
    }
    return t;
}

// Sampler of the wide passes: PAIR = border padding with W >= 2.
template <int PAD, bool PAIR, bool DERIV>
__device__ __forceinline__ Tri wide_sample(const float* __restrict__ M, int D, int H, int W, int x, int y, int z,
                                           float ux, float uy, float uz)
{
    if (PAIR) return sample_pair<DERIV>(M, D, H, W, x, y, z, ux, uy, uz);
    return trilinear<PAD, DERIV>(M, D, H, W, x, y, z, ux, uy, uz);
}

// Pass 1 (SAMPLE: F and Mw staged as floats, the five products formed in
// FP64, exactly, inside the x-window, FP64 sums out) and pass 3 (LOAD: the
// three fp32 fields a, c, e, summed in FP64, fp32 sums out).  A 32 x TY slice
// tile plus an r halo is staged in LDS; the x-window runs over 8 consecutive
// outputs per thread (one fresh sum, then add the entering and subtract the
// leaving tap), the y-window over TY / 16 consecutive rows per thread the
// same way.
template <int NF, bool SAMPLE, int PAD, bool PAIR, int TY>
__global__ void __launch_bounds__(WXT) wide_xy_kernel(WideArgs a, const float* __restrict__ src, void* dstv)
{
    constexpr int Y2M = TY + 2 * WMAXR;
    constexpr int NL = SAMPLE ? 2 : NF;
    typedef typename std::conditional<SAMPLE, double, float>::type Dt;  // stored sums
    Dt* __restrict__ dst = static_cast<Dt*>(dstv);
    __shared__ float P[NL][Y2M * WX2];
    __shared__ double Q[NF][Y2M * WTX];
    const int D = a.D, H = a.H, W = a.W, r = a.r, w = 2 * r + 1;
    const int X2 = WTX + 2 * r, Y2 = TY + 2 * r;
    const size_t N = (size_t)D * H * W;
    const int nty = (H + TY - 1) / TY;
    const int tiles = a.ntx * nty;
    const int z = blockIdx.x / tiles;
    const int t = blockIdx.x - z * tiles;
    const int ty = t / a.ntx, tx = t - ty * a.ntx;
    const int x0 = tx * WTX - r, y0 = ty * TY - r;
    for (int q = threadIdx.x; q < X2 * Y2; q += WXT) {
        const int ly = q / X2, lx = q - ly * X2;
        const int gx = x0 + lx, gy = y0 + ly;
        float v[NL];
#pragma unroll
        for (int c = 0; c < NL; ++c) v[c] = 0.0f;  // zero padding outside the array
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
            const int k = (z * H + gy) * W + gx;
            if (SAMPLE) {
                float ux = 0.f, uy = 0.f, uz = 0.f;
                if (a.u) { ux = a.u[k]; uy = a.u[N + k]; uz = a.u[2 * N + k]; }
                v[0] = a.F[k];
                v[1] = wide_sample<PAD, PAIR, false>(a.M, D, H, W, gx, gy, z, ux, uy, uz).v;
            } else {
#pragma unroll
                for (int c = 0; c < NL; ++c) v[c] = src[c * N + k];
            }
        }
#pragma unroll
        for (int c = 0; c < NL; ++c) P[c][ly * WX2 + lx] = v[c];
    }
    __syncthreads();
    // x-window: row ly, outputs lx0 .. lx0 + 7
    if ((int)threadIdx.x < Y2 * (WTX / WSEG)) {
        const int ly = threadIdx.x / (WTX / WSEG), lx0 = WSEG * (threadIdx.x % (WTX / WSEG));
        auto tap = [&](int lx, double* o) {  // the NF fields at (ly, lx)
            if (SAMPLE) {
                const double f = P[0][ly * WX2 + lx], m = P[NL - 1][ly * WX2 + lx];
                o[0] = f; o[1] = m; o[2] = f * f; o[3] = m * m; o[NF - 1] = f * m;
            } else {
#pragma unroll
                for (int c = 0; c < NF; ++c) o[c] = P[c][ly * WX2 + lx];
            }
        };
        double s[NF], v[NF];
#pragma unroll
        for (int c = 0; c < NF; ++c) s[c] = 0.0;
        for (int d = 0; d < w; ++d) {
            tap(lx0 + d, v);
#pragma unroll
            for (int c = 0; c < NF; ++c) s[c] += v[c];
        }
#pragma unroll
        for (int c = 0; c < NF; ++c) Q[c][ly * WTX + lx0] = s[c];
#pragma unroll
        for (int e = 1; e < WSEG; ++e) {
            double o[NF];
            tap(lx0 + e + w - 1, v);
            tap(lx0 + e - 1, o);
#pragma unroll
            for (int c = 0; c < NF; ++c) {
                s[c] += v[c] - o[c];
                Q[c][ly * WTX + lx0 + e] = s[c];
            }
        }
    }
    __syncthreads();
    // y-window: column lx, rows ly0 .. ly0 + TY / 8 - 1
    constexpr int RY = TY / (WXT / WTX);
    const int lx = threadIdx.x % WTX, ly0 = RY * (threadIdx.x / WTX);
    const int gx = tx * WTX + lx;
    double s[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) s[c] = 0.0;
    for (int d = 0; d < w; ++d)
#pragma unroll
        for (int c = 0; c < NF; ++c) s[c] += Q[c][(ly0 + d) * WTX + lx];
#pragma unroll
    for (int e = 0; e < RY; ++e) {
        if (e > 0)
#pragma unroll
            for (int c = 0; c < NF; ++c) s[c] += Q[c][(ly0 + e + w - 1) * WTX + lx] - Q[c][(ly0 + e - 1) * WTX + lx];
        const int gy = ty * TY + ly0 + e;
        if (gx < W && gy < H) {
            const size_t k = ((size_t)z * H + gy) * W + gx;
#pragma unroll
            for (int c = 0; c < NF; ++c) dst[c * N + k] = (Dt)s[c];
        }
    }
}

// Column of thread (x, y) and the block's z-chunk [z0, z1) in the z passes.
struct WideCol {
    int x, y, z0, z1;
};
__device__ __forceinline__ WideCol wide_col(const WideArgs& a)
{
    int b = blockIdx.x;
    const int cx = b % a.ncx;
    b /= a.ncx;
    const int cy = b % a.ncy, ch = b / a.ncy;
    WideCol c;
    c.x = cx * WCX + (int)threadIdx.x % WCX;
    c.y = cy * WCY + (int)threadIdx.x / WCX;
    c.z0 = ch * a.zchunk;
    c.z1 = min(a.D, c.z0 + a.zchunk);
    return c;
}

// Running z-window sums (FP64) of NF fields at column offset col: s holds
// the sums over slices [z - r, z + r] (clipped to the array) after slide(z).
template <int NF, typename T>
struct ZWindow {
    const T* __restrict__ src;
    size_t N, HW, col;
    int D, r;
    double s[NF];
    __device__ void start(int z)
    {
#pragma unroll
        for (int c = 0; c < NF; ++c) s[c] = 0.0;
        for (int zz = max(z - r, 0); zz <= min(z + r, D - 1); ++zz)
#pragma unroll
            for (int c = 0; c < NF; ++c) s[c] += src[c * N + zz * HW + col];
    }
    __device__ void slide(int z)  // window of z - 1 -> window of z
    {
        const int za = z + r, zr = z - r - 1;
        if (za < D)
#pragma unroll
            for (int c = 0; c < NF; ++c) s[c] += src[c * N + za * HW + col];
        if (zr >= 0)
#pragma unroll
            for (int c = 0; c < NF; ++c) s[c] -= src[c * N + zr * HW + col];
    }
};

// Pass 2: statistics, loss partials, and a, c, e (or the ANTs gradient).
template <int MODE, int PAD>
__global__ void __launch_bounds__(WNT) wide_z_kernel(WideArgs a)
{
    __shared__ double red[WNT];
    const WideCol c = wide_col(a);
    const int D = a.D, H = a.H, W = a.W, r = a.r, w = 2 * r + 1;
    const size_t N = (size_t)D * H * W, HW = (size_t)H * W;
    const double inv = 1.0 / (double)(w * w * w);
    const double gi = a.neg_inv_nroi * (a.grad_scale ? (double)*a.grad_scale : 1.0);
    double lsum = 0.0;
    if (c.x < W && c.y < H && c.z0 < c.z1) {
        const size_t col = (size_t)c.y * W + c.x;
        const bool xyroi = c.y >= a.roi[2] && c.y < a.roi[3] && c.x >= a.roi[4] && c.x < a.roi[5];
        ZWindow<5, double> zw{a.S, N, HW, col, D, r, {}};
        zw.start(c.z0);
        for (int z = c.z0; z < c.z1; ++z) {
            if (z > c.z0) zw.slide(z);
            const bool inroi = xyroi && z >= a.roi[0] && z < a.roi[1];
            const double mf = zw.s[0] * inv, mm = zw.s[1] * inv;
            const double A = fma(-mf, mm, zw.s[4] * inv);
            const double B = fma(-mf, mf, zw.s[2] * inv);
            const double C = fma(-mm, mm, zw.s[3] * inv);
            const double Dn = fma(B, C, a.eps);
            double av = 0.0, cv = 0.0, ev = 0.0;
            if (inroi) {
                lsum += A * A / Dn;
                av = 2.0 * gi * A / Dn;
                cv = av * A * B / Dn;
                ev = fma(cv, mm, -av * mf);
            }
            const size_t k = (size_t)z * HW + col;
            if (MODE == WMODE_BWD) {
                a.E[k] = (float)av;
                a.E[N + k] = (float)cv;
                a.E[2 * N + k] = (float)ev;
            } else if (MODE == WMODE_ANTS) {
                // the derivative of voxel k's own term, without the second window sum
                float g0 = 0.f, g1 = 0.f, g2 = 0.f;
                if (inroi) {
                    float ux = 0.f, uy = 0.f, uz = 0.f;
                    if (a.u) { ux = a.u[k]; uy = a.u[N + k]; uz = a.u[2 * N + k]; }
                    const Tri t = trilinear<PAD, true>(a.M, D, H, W, c.x, c.y, z, ux, uy, uz);
                    const double gm = av * ((double)a.F[k] - mf) - cv * ((double)t.v - mm);
                    g0 = (float)(gm * t.dx);
                    g1 = (float)(gm * t.dy);
                    g2 = (float)(gm * t.dz);
                }
                a.gu[k] = g0;
                a.gu[N + k] = g1;
                a.gu[2 * N + k] = g2;
            }
        }
    }
    const double tot = block_sum<WNT>(lsum, red);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = tot;
}

// Pass 4: z-window of the xy-boxed a, c, e, combined with F_k and Mw_k.
template <int PAD, bool PAIR>
__global__ void __launch_bounds__(WNT) wide_grad_kernel(WideArgs a)
{
    const WideCol c = wide_col(a);
    const int D = a.D, H = a.H, W = a.W, r = a.r, w = 2 * r + 1;
    if (c.x >= W || c.y >= H || c.z0 >= c.z1) return;
    const size_t N = (size_t)D * H * W, HW = (size_t)H * W;
    const double inv = 1.0 / (double)(w * w * w);
    const size_t col = (size_t)c.y * W + c.x;
    ZWindow<3, float> zw{reinterpret_cast<const float*>(a.S), N, HW, col, D, r, {}};
    zw.start(c.z0);
    for (int z = c.z0; z < c.z1; ++z) {
        if (z > c.z0) zw.slide(z);
        const size_t k = (size_t)z * HW + col;
        float ux = 0.f, uy = 0.f, uz = 0.f;
        if (a.u) { ux = a.u[k]; uy = a.u[N + k]; uz = a.u[2 * N + k]; }
        const Tri t = wide_sample<PAD, PAIR, true>(a.M, D, H, W, c.x, c.y, z, ux, uy, uz);
        const double gm = fma((double)a.F[k], zw.s[0], fma(-(double)t.v, zw.s[1], zw.s[2])) * inv;
        a.gu[k] = (float)(gm * t.dx);
        a.gu[N + k] = (float)(gm * t.dy);
        a.gu[2 * N + k] = (float)(gm * t.dz);
    }
}

// loss = 1 - sum(partial) / N_roi, summed in a fixed order
__global__ void __launch_bounds__(256) wide_finalize(const double* __restrict__ partial, int n, double inv_nroi,
                                                     float* loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) *loss = (float)(1.0 - s * inv_nroi);
}

template <int PAD, bool PAIR>
hipError_t wide_run(int mode, const WideArgs& a, const WidePlan& P, hipStream_t st)
{
    const dim3 blk(WNT);
    const long long slices = (long long)a.ntx * a.D;
    const dim3 gs((unsigned)(slices * ((a.H + WTY_S - 1) / WTY_S)));
    const dim3 gl((unsigned)(slices * ((a.H + WTY_L - 1) / WTY_L)));
    const dim3 gz((unsigned)P.nblocks);
    hipLaunchKernelGGL((wide_xy_kernel<5, true, PAD, PAIR, WTY_S>), gs, dim3(WXT), 0, st, a, nullptr,
                       static_cast<void*>(a.S));
    if (mode == WMODE_FWD) hipLaunchKernelGGL((wide_z_kernel<WMODE_FWD, PAD>), gz, blk, 0, st, a);
    else if (mode == WMODE_ANTS) hipLaunchKernelGGL((wide_z_kernel<WMODE_ANTS, PAD>), gz, blk, 0, st, a);
    else {
        hipLaunchKernelGGL((wide_z_kernel<WMODE_BWD, PAD>), gz, blk, 0, st, a);
        hipLaunchKernelGGL((wide_xy_kernel<3, false, PAD, false, WTY_L>), gl, dim3(WXT), 0, st, a, a.E,
                           static_cast<void*>(a.S));
        hipLaunchKernelGGL((wide_grad_kernel<PAD, PAIR>), gz, blk, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace

// z passes: 64 x 4 columns per block, z-chunks of at least 32 slices, about
// 4096 blocks where the volume allows.
WidePlan wide_plan(int D, int H, int W)
{
    WidePlan P;
    P.ncx = (W + WCX - 1) / WCX;
    P.ncy = (H + WCY - 1) / WCY;
    const long long cols = (long long)P.ncx * P.ncy;
    long long want = (4096 + cols - 1) / cols;
    const long long most = max(1, D / 32);
    if (want > most) want = most;
    if (want < 1) want = 1;
    P.zchunk = (int)((D + want - 1) / want);
    P.nchunks = (D + P.zchunk - 1) / P.zchunk;
    P.nblocks = (int)(cols * P.nchunks);
    return P;
}

size_t wide_ws_bytes(int D, int H, int W)
{
    const size_t N = (size_t)D * H * W;
    return 8 * N * sizeof(double) + (size_t)wide_plan(D, H, W).nblocks * sizeof(double);
}

hipError_t lncc_wide_launch(int mode, int win, int pad, const LnccArgs& la, void* ws, float* loss, double nroi,
                            hipStream_t st)
{
    if (win < 11 || win > LNCC_MAX_WINDOW || !(win & 1)) return hipErrorInvalidValue;
    const WidePlan P = wide_plan(la.D, la.H, la.W);
    const size_t N = (size_t)la.D * la.H * la.W;
    WideArgs a;
    a.F = la.F; a.M = la.M; a.u = la.u; a.gu = la.gu; a.grad_scale = la.grad_scale;
    a.S = static_cast<double*>(ws);
    a.E = reinterpret_cast<float*>(a.S + 5 * N);
    a.partial = a.S + 8 * N;
    a.D = la.D; a.H = la.H; a.W = la.W;
    for (int q = 0; q < 6; ++q) a.roi[q] = la.roi[q];
    a.r = (win - 1) / 2;
    a.eps = (double)la.eps;
    a.neg_inv_nroi = -1.0 / nroi;
    a.ntx = (la.W + WTX - 1) / WTX;
    a.ncx = P.ncx; a.ncy = P.ncy; a.zchunk = P.zchunk;
    hipError_t e = pad != PAD_BORDER ? wide_run<PAD_ZEROS, false>(mode, a, P, st)
                   : la.W >= 2        ? wide_run<PAD_BORDER, true>(mode, a, P, st)
                                      : wide_run<PAD_BORDER, false>(mode, a, P, st);
    if (e != hipSuccess || !loss) return e;
    hipLaunchKernelGGL(wide_finalize, dim3(1), dim3(256), 0, st, a.partial, P.nblocks, 1.0 / nroi, loss);
    return hipGetLastError();
}

}  // namespace ffdp
