// BF16 MFMA implicit-GEMM 3x3x3 convolutions (pad 1, stride 1 or 2) for the
// warm-start U-Net, gfx950.  FP32 accumulation.
//
// Activations are channels-last bf16 [N][D][H][W][C].  A convolution input
// may be the channel concatenation of an upsampled coarse tensor xa (nearest
// x2, channels [0, Ca)) and a skip tensor xb (channels [Ca, Ca+Cb)); the
// upsampling and the concatenation happen in the operand gather and are never
// materialised.
//
//   forward      y[o][co] = act(b[co] + sum_{t,ci} X[o*s + t - 1][ci] W[co][t][ci])
//   backward-data dX[i][ci] = sum_{t,co} P[(i + 1 - t)/s][co] W[co][t][ci]
//   backward-weight dW[co][t][ci] = sum_o P[o][co] X[o*s + t - 1][ci]
// with P = dL/dy * act'(y) (LeakyReLU: slope where y <= 0), formed in the
// gather and rounded to bf16 as the MFMA operand.
//
// Forward and backward-data: each 64-lane wave owns one 16-row slab of the
// GEMM (a block of four waves 64 rows) and issues gfx950's
// v_mfma_f32_16x16x32_bf16 over 32-wide K steps.  Operand layout of that
// instruction (lane l, element e):
//   A[i][k]: i = l % 16, k = 8 (l / 16) + e (e < 8)   B[k][j]: k = 8 (l / 16) + e, j = l % 16
//   D[i][j]: i = 4 (l / 16) + e (e < 4), j = l % 16
// K is ordered (tap, channel); a lane's 8 K elements are two groups of 4
// consecutive channels (channel counts are multiples of 4), each one 8-byte
// load of 4 bf16 (or 16 bytes of fp32 for the backward-data operand).  The
// weight operand of 128 K columns for every output column of the block is
// staged in LDS once per block and read by all four waves (rows padded by 8
// bf16 so that the 16 rows a wave reads fall in different banks).
// Backward-weight uses the same instruction with K = output voxels (8
// consecutive voxels per lane).
#include "device.hpp"
#include "internal.hpp"
#include "conv_p.hpp"

namespace ffdp {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // quiet NaN
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);                  // round to nearest even
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ s4v ld4bf(const unsigned short* p)
{
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    s4v r;
    r[0] = (short)(v.x & 0xffffu); r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xffffu); r[3] = (short)(v.y >> 16);
    return r;
}

__device__ __forceinline__ s4v pack4(float a, float b, float c, float d)
{
    s4v r;
    r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
    return r;
}

__device__ __forceinline__ float lrelu_d(unsigned short y, float slope) { return bf2f(y) > 0.0f ? 1.0f : slope; }

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));

// eight bf16 (bit patterns in shorts) as the MFMA operand type
__device__ __forceinline__ bf8v cat8(s4v lo, s4v hi)
{
    const s8v r = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(bf8v, r);
}

// Output-voxel cursor (n, z, y, x) advanced by d voxels without divisions
// (the loop runs about d / W + 1 times).
struct Vox {
    int n, z, y, x;
};
__device__ __forceinline__ Vox vox_of(long long o, int D, int H, int W)
{
    Vox v;
    v.x = (int)(o % W); o /= W;
    v.y = (int)(o % H); o /= H;
    v.z = (int)(o % D);
    v.n = (int)(o / D);
    return v;
}
__device__ __forceinline__ void vox_add(Vox& v, int d, int D, int H, int W)
{
    v.x += d;
    while (v.x >= W) {
        v.x -= W;
        if (++v.y == H) {
            v.y = 0;
            if (++v.z == D) { v.z = 0; ++v.n; }
        }
    }
}

constexpr int CONV_KC = 128;            // K columns of the weight tile staged per round
constexpr int CONV_KCP = CONV_KC + 8;   // LDS row pitch (bf16)

// Stage rows [0, 16 NT) x columns [k0, k0 + KC) of a row-major bf16 weight
// matrix wsrc [rows][K] into LDS (zeros outside rows < nrows, k < K).  Rows
// start 8-byte aligned (K is a multiple of 4), so each thread moves 4 bf16
// per load.
template <int NT>
__device__ __forceinline__ void stage_weights(unsigned short* __restrict__ ws, const unsigned short* __restrict__ wsrc,
                                              int nrows, int K, int k0)
{
    constexpr int Q = NT * 16 * (CONV_KC / 4);  // 4-element groups
    for (int q = threadIdx.x; q < Q; q += 256) {
        const int r = q / (CONV_KC / 4), c = (q - r * (CONV_KC / 4)) * 4;
        uint2 v = make_uint2(0u, 0u);
        if (r < nrows && k0 + c < K) v = *reinterpret_cast<const uint2*>(wsrc + (size_t)r * K + k0 + c);
        *reinterpret_cast<uint2*>(ws + r * CONV_KCP + c) = v;
    }
}

// B operand of one K step from the staged tile: column j of tile jt, K rows
// kk + 8 (l / 16) .. + 8
__device__ __forceinline__ bf8v b_from_lds(const unsigned short* __restrict__ ws, int jt, int lane, int kk)
{
    const uint4 v = *reinterpret_cast<const uint4*>(ws + (jt * 16 + (lane & 15)) * CONV_KCP + kk + (lane >> 4) * 8);
    return __builtin_bit_cast(bf8v, v);
}

// ---------------------------------------------------------------- forward --
// C8: Ca and Cb are multiples of 8, so a lane's 8 K elements are 8
// contiguous channels of one tap and one 16-byte load.  MT: output tiles of
// 16 voxels per wave; each B operand read from LDS feeds MT MFMAs (with one
// voxel tile per wave the LDS reads of the weights, one per MFMA, bound the
// kernel).
template <int NT, bool C8, int MT>
__global__ void __launch_bounds__(256) conv_fwd_kernel(ConvGeom g, const unsigned short* __restrict__ xa,
                                                       const unsigned short* __restrict__ xb,
                                                       const unsigned short* __restrict__ w,
                                                       const float* __restrict__ bias, int act, float slope,
                                                       unsigned short* __restrict__ ybf, float* __restrict__ yf)
{
    __shared__ __attribute__((aligned(16))) unsigned short ws[NT * 16 * CONV_KCP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Cin = g.Ca + g.Cb;
    const int K = 27 * Cin;
    const long long M = (long long)g.N * g.Do * g.Ho * g.Wo;
    const long long mb = ((long long)blockIdx.x * 4 + wave) * 16 * MT;  // the wave's first output voxel
    int n[MT], zs[MT], ys[MT], xs[MT];  // each row's input corner (tap 0, 0, 0)
    bool mvalid[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const long long m = mb + 16 * mt + (lane & 15);
        mvalid[mt] = m < M;
        n[mt] = 0; zs[mt] = 0; ys[mt] = 0; xs[mt] = 0;
        if (mvalid[mt]) {
            const Vox v = vox_of(m, g.Do, g.Ho, g.Wo);
            n[mt] = v.n;
            zs[mt] = v.z * g.stride - 1; ys[mt] = v.y * g.stride - 1; xs[mt] = v.x * g.stride - 1;
        }
    }
    const int Da = g.Di >> 1, Ha = g.Hi >> 1, Wa = g.Wi >> 1;
    auto load_a4 = [&](int mt, int t, int c) {  // channels c..c+3 of tap t (32-bit voxel indices)
        s4v a = s4v{0, 0, 0, 0};
        const int dz = t / 9, dy = (t - 9 * dz) / 3, dx = t - 9 * dz - 3 * dy;
        const int zi = zs[mt] + dz, yi = ys[mt] + dy, xi = xs[mt] + dx;
        if (mvalid[mt] && t < 27 && (unsigned)zi < (unsigned)g.Di && (unsigned)yi < (unsigned)g.Hi &&
            (unsigned)xi < (unsigned)g.Wi) {
            if (c < g.Ca) {
                const unsigned v = g.ups ? ((unsigned)(n[mt] * Da + (zi >> 1)) * Ha + (yi >> 1)) * Wa + (xi >> 1)
                                         : ((unsigned)(n[mt] * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                a = ld4bf(xa + (size_t)v * g.Ca + c);
            } else {
                const unsigned v = ((unsigned)(n[mt] * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                a = ld4bf(xb + (size_t)v * g.Cb + (c - g.Ca));
            }
        }
        return a;
    };
    auto load_a8 = [&](int mt, int t, int c) {  // channels c..c+7 of tap t (C8)
        uint4 a = make_uint4(0u, 0u, 0u, 0u);
        const int dz = t / 9, dy = (t - 9 * dz) / 3, dx = t - 9 * dz - 3 * dy;
        const int zi = zs[mt] + dz, yi = ys[mt] + dy, xi = xs[mt] + dx;
        if (mvalid[mt] && t < 27 && (unsigned)zi < (unsigned)g.Di && (unsigned)yi < (unsigned)g.Hi &&
            (unsigned)xi < (unsigned)g.Wi) {
            if (c < g.Ca) {
                const unsigned v = g.ups ? ((unsigned)(n[mt] * Da + (zi >> 1)) * Ha + (yi >> 1)) * Wa + (xi >> 1)
                                         : ((unsigned)(n[mt] * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                a = *reinterpret_cast<const uint4*>(xa + (size_t)v * g.Ca + c);
            } else {
                const unsigned v = ((unsigned)(n[mt] * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                a = *reinterpret_cast<const uint4*>(xb + (size_t)v * g.Cb + (c - g.Ca));
            }
        }
        return __builtin_bit_cast(bf8v, a);
    };
    const int kg = (lane >> 4) * 8;
    // the lane's K index k = (tap t, channel c), advanced by 32 per step
    int t = kg / Cin, c = kg - t * Cin;
    f4v acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[mt][j] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += CONV_KC) {
        __syncthreads();
        stage_weights<NT>(ws, w, g.Cout, K, k0);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < CONV_KC; kk += 32) {
            if (k0 + kk >= K) break;  // uniform: no all-zero K steps in the last round
            bf8v a[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                if (C8) {
                    a[mt] = load_a8(mt, t, c);
                } else {
                    const bool wrap = c + 4 >= Cin;  // channels c + 4 .. c + 7 start the next tap (Cin % 4 == 0)
                    a[mt] = cat8(load_a4(mt, t, c), load_a4(mt, wrap ? t + 1 : t, wrap ? c + 4 - Cin : c + 4));
                }
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const bf8v b = b_from_lds(ws, j, lane, kk);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[mt][j], 0, 0, 0);
            }
            c += 32;
            while (c >= Cin) { c -= Cin; ++t; }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long long mo = mb + 16 * mt + (lane >> 4) * 4 + e;
                if (mo < M && co < g.Cout) {
                    float v = acc[mt][j][e] + (bias ? bias[co] : 0.0f);
                    if (act) v = v > 0.0f ? v : v * slope;
                    if (ybf) ybf[mo * g.Cout + co] = f2bf(v);
                    if (yf) yf[mo * g.Cout + co] = v;
                }
            }
        }
}

// ----------------------------------------------------------- backward data --
// dX over the virtual (concatenated, fine-resolution) input, fp32 [N][Di][Hi][Wi][Cin];
// accumulate = 1 adds to dX.  wt is the weight in [Cin][27][Cout] order.
// C8: Cout is a multiple of 8, so a lane's 8 K elements are 8 contiguous
// output channels of one tap (two 16-byte loads of dL/dy, one of y).
// PAR (stride 2): an input voxel i receives tap d along an axis only where
// i + 1 - d is even (d = 1 for even i, d = 0 or 2 for odd i), so the input
// voxels are split into the 8 parity classes of (z, y, x) and a block takes
// 64 voxels of one class: its K runs over that class's 1 to 8 taps instead
// of all 27 (3.375 on average), and no product is a structural zero.
// PB: P = dL/dy act'(y) arrives precomputed as bf16 in dL/dy's layout (pb),
// so a lane's 8 K elements are one 16-byte load (4 channels: 8 bytes) and no
// conversion; dy and y are not read.
template <int NT, bool C8, bool PAR, bool PB, int MT>
__global__ void __launch_bounds__(256) conv_bwd_data_kernel(ConvGeom g, const float* __restrict__ dy,
                                                            const unsigned short* __restrict__ y, float slope,
                                                            const unsigned short* __restrict__ pb,
                                                            const unsigned short* __restrict__ wt,
                                                            float* __restrict__ dx, int accumulate)
{
    __shared__ __attribute__((aligned(16))) unsigned short ws[NT * 16 * CONV_KCP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Cin = g.Ca + g.Cb;
    const long long M = (long long)g.N * g.Di * g.Hi * g.Wi;
    // parity class (PAR): bits 2, 1, 0 = z, y, x parity; rows index the class's
    // voxels over the half-resolution grid Dc x Hc x Wc (rounded up)
    const int Dc = (g.Di + 1) >> 1, Hc = (g.Hi + 1) >> 1, Wc = (g.Wi + 1) >> 1;
    const long long Mc = (long long)g.N * Dc * Hc * Wc;
    const int bpc = PAR ? (int)((Mc + 64 * MT - 1) / (64 * MT)) : 0;  // blocks per class
    const int cls = PAR ? (int)blockIdx.x / bpc : 0;
    const int pz = (cls >> 2) & 1, py = (cls >> 1) & 1, px = cls & 1;
    const int ny = PAR ? 1 + py : 3, nx = PAR ? 1 + px : 3;  // taps per axis
    const int ntap = PAR ? (1 + pz) * ny * nx : 27;
    const int K = ntap * g.Cout;
    // the wave's MT tiles of 16 rows
    const long long m0 = ((long long)(PAR ? (int)blockIdx.x - cls * bpc : (int)blockIdx.x) * 4 + wave) * 16 * MT;
    auto voxel = [&](long long r, int& n_, int& z_, int& y_, int& x_) -> bool {  // row -> voxel
        if (!PAR) {
            if (r >= M) return false;
            const Vox v = vox_of(r, g.Di, g.Hi, g.Wi);
            n_ = v.n; z_ = v.z; y_ = v.y; x_ = v.x;
            return true;
        }
        if (r >= Mc) return false;
        const Vox v = vox_of(r, Dc, Hc, Wc);
        n_ = v.n; z_ = 2 * v.z + pz; y_ = 2 * v.y + py; x_ = 2 * v.x + px;
        return z_ < g.Di && y_ < g.Hi && x_ < g.Wi;
    };
    int n[MT], zi[MT], yi[MT], xi[MT];
    bool mvalid[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        n[mt] = 0; zi[mt] = 0; yi[mt] = 0; xi[mt] = 0;
        mvalid[mt] = voxel(m0 + 16 * mt + (lane & 15), n[mt], zi[mt], yi[mt], xi[mt]);
    }
    // tap number of the class's j-th tap (PAR), else j itself
    auto tap_of = [&](int j) -> int {
        if (!PAR) return j;
        const int jz = j / (ny * nx), jr = j - jz * ny * nx, jy = jr / nx, jx = jr - jy * nx;
        const int dz = pz ? 2 * jz : 1, dyy = py ? 2 * jy : 1, dx_ = px ? 2 * jx : 1;
        return dz * 9 + dyy * 3 + dx_;
    };
    // element offset of P at output channel co of tap t, or -1 where the tap
    // reaches no output voxel (a non-integer or out-of-range output index)
    auto p_offset = [&](int mt, int j, int co) -> long long {  // j: tap index within the class (PAR) or tap
        if (!mvalid[mt] || j >= ntap) return -1;
        const int t = tap_of(j);
        const int dz = t / 9, dyy = (t - 9 * dz) / 3, dx_ = t - 9 * dz - 3 * dyy;
        int oz = zi[mt] + 1 - dz, oy = yi[mt] + 1 - dyy, ox = xi[mt] + 1 - dx_;
        bool ok = oz >= 0 && oy >= 0 && ox >= 0;
        if (g.stride == 2) {
            ok = ok && !(oz & 1) && !(oy & 1) && !(ox & 1);
            oz >>= 1; oy >>= 1; ox >>= 1;
        }
        ok = ok && oz < g.Do && oy < g.Ho && ox < g.Wo;
        return ok ? (long long)(((unsigned)(n[mt] * g.Do + oz) * g.Ho + oy) * g.Wo + ox) * g.Cout + co : -1;
    };
    auto load_p4 = [&](int mt, int t, int co) {  // P = dL/dy * act'(y) at output channels co..co+3 of tap t
        s4v a = s4v{0, 0, 0, 0};
        const long long o = p_offset(mt, t, co);
        if (PB) {
            if (o >= 0) a = ld4bf(pb + o);
        } else if (o >= 0) {
            const float4 d4 = *reinterpret_cast<const float4*>(dy + o);
            float f[4] = {1.f, 1.f, 1.f, 1.f};
            if (y) {
                const s4v yv = ld4bf(y + o);
#pragma unroll
                for (int q = 0; q < 4; ++q) f[q] = lrelu_d((unsigned short)yv[q], slope);
            }
            a = pack4(d4.x * f[0], d4.y * f[1], d4.z * f[2], d4.w * f[3]);
        }
        return a;
    };
    auto load_p8 = [&](int mt, int t, int co) {  // channels co..co+7 of tap t (C8)
        s4v lo = s4v{0, 0, 0, 0}, hi = s4v{0, 0, 0, 0};
        const long long o = p_offset(mt, t, co);
        if (PB) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (o >= 0) v = *reinterpret_cast<const uint4*>(pb + o);
            return __builtin_bit_cast(bf8v, v);
        }
        if (o >= 0) {
            const float4 d0 = *reinterpret_cast<const float4*>(dy + o);
            const float4 d1 = *reinterpret_cast<const float4*>(dy + o + 4);
            float f[8] = {1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f, 1.f};
            if (y) {
                const uint4 yv = *reinterpret_cast<const uint4*>(y + o);
                const unsigned yw[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
                for (int q = 0; q < 8; ++q) f[q] = lrelu_d((unsigned short)(yw[q >> 1] >> (16 * (q & 1))), slope);
            }
            lo = pack4(d0.x * f[0], d0.y * f[1], d0.z * f[2], d0.w * f[3]);
            hi = pack4(d1.x * f[4], d1.y * f[5], d1.z * f[6], d1.w * f[7]);
        }
        return cat8(lo, hi);
    };
    const int kg = (lane >> 4) * 8;
    // the lane's K index k = (tap t, output channel c), advanced by 32 per step
    int t = kg / g.Cout, c = kg - t * g.Cout;
    f4v acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[mt][j] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += CONV_KC) {
        __syncthreads();
        if (PAR) {
            // the class's K columns (j, c) from wt [Cin][27][Cout]: groups of 4
            // channels of one tap (Cout % 4 == 0) are contiguous there
            constexpr int Q = NT * 16 * (CONV_KC / 4);
            const int K27 = 27 * g.Cout;
            for (int q = threadIdx.x; q < Q; q += 256) {
                const int r = q / (CONV_KC / 4), cc = (q - r * (CONV_KC / 4)) * 4;
                uint2 v = make_uint2(0u, 0u);
                const int k = k0 + cc;
                if (r < Cin && k < K) {
                    const int j = k / g.Cout, c4 = k - j * g.Cout;
                    v = *reinterpret_cast<const uint2*>(wt + (size_t)r * K27 + tap_of(j) * g.Cout + c4);
                }
                *reinterpret_cast<uint2*>(ws + r * CONV_KCP + cc) = v;
            }
        } else {
            stage_weights<NT>(ws, wt, Cin, K, k0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < CONV_KC; kk += 32) {
            if (k0 + kk >= K) break;  // uniform: past the last K column
            bf8v a[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                if (C8) {
                    a[mt] = load_p8(mt, t, c);
                } else {
                    const bool wrap = c + 4 >= g.Cout;  // Cout % 4 == 0
                    a[mt] = cat8(load_p4(mt, t, c), load_p4(mt, wrap ? t + 1 : t, wrap ? c + 4 - g.Cout : c + 4));
                }
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const bf8v b = b_from_lds(ws, j, lane, kk);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[mt][j], 0, 0, 0);
            }
            c += 32;
            while (c >= g.Cout) { c -= g.Cout; ++t; }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        long long vo[4];  // voxels of the lane's 4 output rows of tile mt (-1: none)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int n_, z_, y_, x_;
            const long long r = m0 + 16 * mt + (lane >> 4) * 4 + e;
            vo[e] = -1;
            if (voxel(r, n_, z_, y_, x_)) vo[e] = PAR ? (((long long)n_ * g.Di + z_) * g.Hi + y_) * g.Wi + x_ : r;
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int ci = j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (vo[e] >= 0 && ci < Cin) {
                    float* p = dx + vo[e] * Cin + ci;
                    *p = accumulate ? *p + acc[mt][j][e] : acc[mt][j][e];
                }
            }
        }
    }
}

// --------------------------------------------------------- backward weight --
// P^T = bf16(dL/dy act'(y)) in [Cout][MP] order (MP = M rounded up to 8,
// zeros past M) for the voxel-chunk weight-gradient kernels: their MFMA A
// operand, 8 consecutive output voxels of one channel, is then one aligned
// 16-byte load.  A block transposes 64 voxels x Cout channels through LDS
// (coalesced reads along channels, coalesced writes along voxels).  The
// rounding is that of the operand packing (round to nearest even).
constexpr int PT_MAXC = 128;
__global__ void __launch_bounds__(256) p_transpose_kernel(const float* __restrict__ dy,
                                                          const unsigned short* __restrict__ y, float slope,
                                                          const unsigned short* __restrict__ pbf, long long M,
                                                          int Cout, long long MP, unsigned short* __restrict__ pt)
{
    __shared__ unsigned short tile[PT_MAXC][64 + 2];
    const long long o0 = (long long)blockIdx.x * 64;
    const long long nv = min(64LL, M - o0);  // <= 0 in the padding past M
    for (int q = threadIdx.x; q < 64 * Cout; q += 256) {
        const int v = q / Cout, co = q - v * Cout;
        unsigned short h = 0;  // bf16 zero
        if (v < nv) {
            const size_t k = (size_t)(o0 + v) * Cout + co;
            if (pbf) {
                h = pbf[k];
            } else {
                float p = dy[k];
                if (y) p *= lrelu_d(y[k], slope);
                h = f2bf(p);
            }
        }
        tile[co][v] = h;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < Cout * 64; q += 256) {
        const int co = q >> 6, v = q & 63;
        if (o0 + v < MP) pt[(size_t)co * MP + o0 + v] = tile[co][v];
    }
}

// A operand of output channel co for the 8 output voxels o .. o + 7 (o a
// multiple of 8): one 16-byte load of P^T, the voxels at or past oe zeroed.
__device__ __forceinline__ bf8v load_pt8(const unsigned short* __restrict__ pt, long long MP, int co, int Cout,
                                         long long o, long long oe)
{
    s8v r = s8v{0, 0, 0, 0, 0, 0, 0, 0};
    if (co < Cout && o < oe) {
        r = *reinterpret_cast<const s8v*>(pt + (size_t)co * MP + o);
        if (o + 8 > oe)
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (o + e >= oe) r[e] = 0;
    }
    return __builtin_bit_cast(bf8v, r);
}

// Block (chunk, tap t): partial dW[co][t][ci] over output voxels
// [chunk*VC, chunk*VC + VC), written to part[chunk][co][t][ci].  Wave w owns
// the ci-tiles w, w+4, ... and all co-tiles.  GEMM rows co, columns ci, K =
// output voxels: each lane takes 8 consecutive output voxels per 32-wide K
// step of v_mfma_f32_16x16x32_bf16.
template <int TM, int TNW>
__global__ void __launch_bounds__(256) conv_bwd_weight_kernel(ConvGeom g, const unsigned short* __restrict__ xa,
                                                              const unsigned short* __restrict__ xb,
                                                              const unsigned short* __restrict__ pt, long long MP,
                                                              long long VC, float* __restrict__ part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Cin = g.Ca + g.Cb;
    const int t = blockIdx.y;
    const int dz = t / 9, dyy = (t / 3) % 3, dx_ = t % 3;
    const long long M = (long long)g.N * g.Do * g.Ho * g.Wo;
    const long long ob = (long long)blockIdx.x * VC;
    const long long oe = min(M, ob + VC);
    const int TN = (Cin + 15) / 16;
    f4v acc[TM][TNW];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TNW; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    const int kg = (lane >> 4) * 8;
    Vox cur = vox_of(ob + kg, g.Do, g.Ho, g.Wo);  // the lane's first voxel of the K step
    for (long long o0 = ob; o0 < oe; o0 += 32) {
        // this lane's 8 output voxels o0 + kg + e and their shifted input voxels
        long long iv[8], iva[8];  // input voxel; its coarse voxel where part a is upsampled
        bool ov[8], iok[8];
        Vox v = cur;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (e) vox_add(v, 1, g.Do, g.Ho, g.Wo);
            const long long o = o0 + kg + e;
            ov[e] = o < oe;
            iok[e] = false;
            iv[e] = 0;
            iva[e] = 0;
            if (ov[e]) {
                const int zi = v.z * g.stride + dz - 1, yi = v.y * g.stride + dyy - 1, xi = v.x * g.stride + dx_ - 1;
                iok[e] = (unsigned)zi < (unsigned)g.Di && (unsigned)yi < (unsigned)g.Hi && (unsigned)xi < (unsigned)g.Wi;
                iv[e] = (((long long)v.n * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                if (g.ups)
                    iva[e] = (((long long)v.n * (g.Di >> 1) + (zi >> 1)) * (g.Hi >> 1) + (yi >> 1)) * (g.Wi >> 1) +
                             (xi >> 1);
            }
        }
        vox_add(cur, 32, g.Do, g.Ho, g.Wo);
        // A operands: P[o][co] for the co-tiles
        bf8v a[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = load_pt8(pt, MP, i * 16 + (lane & 15), g.Cout, o0 + kg, oe);
#pragma unroll
        for (int jj = 0; jj < TNW; ++jj) {
            const int jt = wave + 4 * jj;
            if (jt >= TN) break;
            const int ci = jt * 16 + (lane & 15);
            s8v bs;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                unsigned short h = 0;
                if (iok[e] && ci < Cin) {
                    const long long v = iv[e];
                    if (ci < g.Ca) {
                        if (g.ups) {
                            h = xa[(size_t)iva[e] * g.Ca + ci];
                        } else {
                            h = xa[(size_t)v * g.Ca + ci];
                        }
                    } else {
                        h = xb[(size_t)v * g.Cb + (ci - g.Ca)];
                    }
                }
                bs[e] = (short)h;
            }
            const bf8v b = __builtin_bit_cast(bf8v, bs);
#pragma unroll
            for (int i = 0; i < TM; ++i) acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][jj], 0, 0, 0);
        }
    }
    // D[i = co][j = ci]: lane holds co = 16 i_t + 4 (l/16) + e, ci = 16 jt + l % 16
    float* P = part + (size_t)blockIdx.x * g.Cout * 27 * Cin;
#pragma unroll
    for (int jj = 0; jj < TNW; ++jj) {
        const int jt = wave + 4 * jj;
        if (jt >= TN) break;
        const int ci = jt * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = i * 16 + (lane >> 4) * 4 + e;
                if (co < g.Cout && ci < Cin) P[((size_t)co * 27 + t) * Cin + ci] = acc[i][jj][e];
            }
    }
}

// Backward-weight for layers with few channels (TM * TN <= 3 tiles: the
// full-resolution layers): a block takes a chunk of output voxels for all 27
// taps, and wave w accumulates taps w, w + 4, ... (7 or 6 of them), so P =
// dL/dy act'(y) of a K step is loaded once per wave for all of its taps
// (the tap-per-block kernel reads it once per tap, which dominates when the
// channel counts are small).  part[chunk][co][t][ci] as conv_bwd_weight_kernel.
template <int TM, int TN>
__global__ void __launch_bounds__(256) conv_bwd_weight_taps_kernel(ConvGeom g, const unsigned short* __restrict__ xa,
                                                                   const unsigned short* __restrict__ xb,
                                                                   const unsigned short* __restrict__ pt,
                                                                   long long MP, long long VC,
                                                                   float* __restrict__ part)
{
    constexpr int QT = 7;  // taps per wave: 27 = 4 * 7 - 1
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Cin = g.Ca + g.Cb;
    const long long M = (long long)g.N * g.Do * g.Ho * g.Wo;
    const long long ob = (long long)blockIdx.x * VC;
    const long long oe = min(M, ob + VC);
    const int Da = g.Di >> 1, Ha = g.Hi >> 1, Wa = g.Wi >> 1;
    f4v acc[QT][TM][TN];
#pragma unroll
    for (int q = 0; q < QT; ++q)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[q][i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    const int kg = (lane >> 4) * 8;
    Vox cur = vox_of(ob + kg, g.Do, g.Ho, g.Wo);  // the lane's first voxel of the K step
    for (long long o0 = ob; o0 < oe; o0 += 32) {
        // the lane's 8 output voxels o0 + kg + e: batch index and the input
        // corner (tap 0, 0, 0) of each
        int vn[8], vz[8], vy[8], vx[8];
        bool ov[8];
        Vox v = cur;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (e) vox_add(v, 1, g.Do, g.Ho, g.Wo);
            const long long o = o0 + kg + e;
            ov[e] = o < oe;
            vn[e] = ov[e] ? v.n : 0;
            vz[e] = v.z * g.stride - 1; vy[e] = v.y * g.stride - 1; vx[e] = v.x * g.stride - 1;
        }
        vox_add(cur, 32, g.Do, g.Ho, g.Wo);
        bf8v a[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = load_pt8(pt, MP, i * 16 + (lane & 15), g.Cout, o0 + kg, oe);
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            const int t = wave + 4 * q;
            if (t >= 27) break;
            const int dz = t / 9, dyy = (t / 3) % 3, dx_ = t % 3;
            bf8v b[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int ci = j * 16 + (lane & 15);
                s8v bs;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int zi = vz[e] + dz, yi = vy[e] + dyy, xi = vx[e] + dx_;
                    unsigned short h = 0;
                    if (ov[e] && ci < Cin && (unsigned)zi < (unsigned)g.Di && (unsigned)yi < (unsigned)g.Hi &&
                        (unsigned)xi < (unsigned)g.Wi) {
                        if (ci < g.Ca) {
                            const size_t va = g.ups ? (((size_t)vn[e] * Da + (zi >> 1)) * Ha + (yi >> 1)) * Wa + (xi >> 1)
                                                    : (((size_t)vn[e] * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                            h = xa[va * g.Ca + ci];
                        } else {
                            const size_t vb = (((size_t)vn[e] * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                            h = xb[vb * g.Cb + (ci - g.Ca)];
                        }
                    }
                    bs[e] = (short)h;
                }
                b[j] = __builtin_bit_cast(bf8v, bs);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[q][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[q][i][j], 0, 0, 0);
        }
    }
    float* P = part + (size_t)blockIdx.x * g.Cout * 27 * Cin;
#pragma unroll
    for (int q = 0; q < QT; ++q) {
        const int t = wave + 4 * q;
        if (t >= 27) break;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int ci = j * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = i * 16 + (lane >> 4) * 4 + e;
                    if (co < g.Cout && ci < Cin) P[((size_t)co * 27 + t) * Cin + ci] = acc[q][i][j][e];
                }
        }
    }
}

// Backward-weight of the stride-1 layers with Cout <= 64, staged in LDS.  A
// block takes one tap plane dz and one chunk of 4 NG input channels, and walks
// a chunk of steps along y: a step is YB rows of 30 consecutive output voxels
// along x at one (n, z), rows y0 .. y0 + YB - 1, whose taps read the 32
// input voxels x0 - 1 .. x0 + 30 of the rows y0 - 1 .. y0 + YB.  LDS holds
//   Xs[c][slot][k]       input row yi in slot (yi + 1) % (YB + 2), k = xi - x0 + 1
//   Ps[dx][co][j][k]     = bf16(P[row y0 + j, x0 + k - dx][co]) (0 outside)
// so that the product for tap (dy, dx) and row j is
// sum_k Ps[dx][co][j][k] Xs[c][slot(y0 + j + dy - 1)][k], and every MFMA
// operand is one aligned 16-byte LDS read (8 consecutive k: the K layout of
// v_mfma_f32_16x16x32_bf16).  Walking along y, a step stages YB new input
// rows (YB + 2 at the start of a run) and P; the global loads of the next
// step are in flight during the MFMAs of the current one.  Wave w
// accumulates the work items w, w+4, ... of the 9 (dy, dx) taps x NG/4
// channel tiles x TM output-channel tiles.  part[chunk][co][t][ci] as
// conv_bwd_weight_kernel.
constexpr int WR_KP = 40;   // LDS row pitch (bf16): 32 voxels + 8
constexpr int WR_SEG = 30;  // output voxels per row of a step
__host__ __device__ constexpr int wgrad_rows_yb(int tm) { return tm == 1 ? 4 : (tm == 2 ? 2 : 1); }
template <int TM, int NG, bool PB>
__global__ void __launch_bounds__(256) conv_wgrad_rows_kernel(ConvGeom g, const unsigned short* __restrict__ xa,
                                                              const unsigned short* __restrict__ xb,
                                                              const float* __restrict__ dy,
                                                              const unsigned short* __restrict__ y, float slope,
                                                              const unsigned short* __restrict__ pbf, long long VS,
                                                              float* __restrict__ part)
{
    constexpr int YB = wgrad_rows_yb(TM);  // output rows per step
    constexpr int R = YB + 2;              // ring slots of input rows
    constexpr int CC = 4 * NG;             // channels per block (whole 16-channel tiles)
    constexpr int NT = NG / 4;             // channel tiles
    constexpr int NI = 9 * NT * TM;        // work items per block
    constexpr int QI = (NI + 3) / 4;       // per wave
    constexpr int XPT = (R * 2 * NT + 3) / 4;  // staging wave-items per wave (a run start)
    constexpr int NP = YB * WR_SEG * TM * 4;   // P loads: rows x 30 voxels x 4-channel groups
    constexpr int NPT = (NP + 255) / 256;
    __shared__ __attribute__((aligned(16))) unsigned short Xs[CC * R * WR_KP];
    __shared__ __attribute__((aligned(16))) unsigned short Ps[3 * TM * 16 * YB * WR_KP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Cin = g.Ca + g.Cb;
    const int nsx = (g.Wo + WR_SEG - 1) / WR_SEG, nyb = (g.Ho + YB - 1) / YB;
    const long long S = (long long)g.N * g.Do * nsx * nyb;
    const int dz = blockIdx.y % 3, c0 = (blockIdx.y / 3) * CC;
    const int ncv = min(CC, Cin - c0);  // valid channels of this chunk
    const long long sb = (long long)blockIdx.x * VS, se = min(S, sb + VS);
    const int Da = g.Di >> 1, Ha = g.Hi >> 1, Wa = g.Wi >> 1;
    const int kxl = lane & 15, cgl = lane >> 4;
    // P slots never written (k = 30, 31 for dx = 0; 0, 31 for dx = 1; 0, 1
    // for dx = 2) stay zero
    for (int i = threadIdx.x; i < 3 * TM * 16 * YB * WR_KP / 2; i += 256) reinterpret_cast<unsigned*>(Ps)[i] = 0u;
    __syncthreads();
    f4v acc[QI];
#pragma unroll
    for (int q = 0; q < QI; ++q) acc[q] = f4v{0.f, 0.f, 0.f, 0.f};
    // global loads of one step's operands into registers, raw (xr: 4 bf16
    // channels of X; dr, yr: dL/dy and y, or yr: P in bf16 when PB)
    uint2 xr[XPT], yr[NPT];
    float4 dr[NPT];
    int nrow_ld = 0, row0_ld = 0, y0_ld = 0;  // staged rows yi = y0 + row0 + r, r < nrow
    // coordinates of the next step to load, advanced without divisions
    int yb, xs, zo, n;
    {
        long long q = sb;
        yb = (int)(q % nyb); q /= nyb;
        xs = (int)(q % nsx); q /= nsx;
        zo = (int)(q % g.Do);
        n = (int)(q / g.Do);
    }
    bool first = true;
    auto load_step = [&]() {
        const int x0 = xs * WR_SEG, y0 = yb * YB;
        const int zi = zo + dz - 1;
        const bool run = first || yb == 0;  // a new run along y: YB + 2 rows
        nrow_ld = run ? R : YB;
        row0_ld = run ? -1 : 1;
        y0_ld = y0;
        const bool zok = (unsigned)zi < (unsigned)g.Di;
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int wi = wave + 4 * u;
            const int r = wi / (2 * NT), kxc = (wi / NT) % 2, ct = wi % NT;
            const int xi = x0 - 1 + 16 * kxc + kxl, yi = y0 + row0_ld + r;
            const int c = c0 + 16 * ct + 4 * cgl;
            xr[u] = make_uint2(0u, 0u);
            if (r < nrow_ld && zok && c - c0 < ncv && (unsigned)xi < (unsigned)g.Wi && (unsigned)yi < (unsigned)g.Hi) {
                const unsigned short* src;
                if (c < g.Ca) {
                    const size_t va = g.ups ? (((size_t)n * Da + (zi >> 1)) * Ha + (yi >> 1)) * Wa + (xi >> 1)
                                            : (((size_t)n * g.Di + zi) * g.Hi + yi) * g.Wi + xi;
                    src = xa + va * g.Ca + c;
                } else {
                    src = xb + ((((size_t)n * g.Di + zi) * g.Hi + yi) * g.Wi + xi) * g.Cb + (c - g.Ca);
                }
                xr[u] = *reinterpret_cast<const uint2*>(src);
            }
        }
        const size_t oplane = ((size_t)n * g.Do + zo) * g.Ho;
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int it = threadIdx.x + 256 * u;
            const int cg = (it % (TM * 4)) * 4, rest = it / (TM * 4);
            const int jx = rest % WR_SEG, jy = rest / WR_SEG;
            dr[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            yr[u] = PB ? make_uint2(0u, 0u) : make_uint2(0x3f803f80u, 0x3f803f80u);  // y = 1: no activation factor
            if (it < NP && x0 + jx < g.Wo && y0 + jy < g.Ho && cg < g.Cout) {  // Cout is a multiple of 4
                const size_t o = ((oplane + y0 + jy) * g.Wo + x0 + jx) * g.Cout + cg;
                if (PB) {
                    yr[u] = *reinterpret_cast<const uint2*>(pbf + o);
                } else {
                    dr[u] = *reinterpret_cast<const float4*>(dy + o);
                    if (y) yr[u] = *reinterpret_cast<const uint2*>(y + o);
                }
            }
        }
        first = false;
        if (++yb == nyb) {
            yb = 0;
            if (++xs == nsx) {
                xs = 0;
                if (++zo == g.Do) { zo = 0; ++n; }
            }
        }
    };
    if (sb < se) load_step();
    for (long long sg = sb; sg < se; ++sg) {
        const int y0 = y0_ld;  // this step's first row
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int it = threadIdx.x + 256 * u;
            if (it >= NP) break;
            const int cg = (it % (TM * 4)) * 4, rest = it / (TM * 4);
            const int jx = rest % WR_SEG, jy = rest / WR_SEG;
            const float pv[4] = {dr[u].x, dr[u].y, dr[u].z, dr[u].w};
            const unsigned short yv[4] = {(unsigned short)(yr[u].x & 0xffffu), (unsigned short)(yr[u].x >> 16),
                                          (unsigned short)(yr[u].y & 0xffffu), (unsigned short)(yr[u].y >> 16)};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const unsigned short h = PB ? yv[c] : f2bf(pv[c] * lrelu_d(yv[c], slope));
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) Ps[(((dx * TM * 16 + cg + c) * YB) + jy) * WR_KP + jx + dx] = h;
            }
        }
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int wi = wave + 4 * u;
            const int r = wi / (2 * NT), kxc = (wi / NT) % 2, ct = wi % NT;
            if (r >= nrow_ld) break;
            const int slot = (y0 + row0_ld + r + 1) % R;  // input row y0 + row0 + r
            unsigned short* dst = Xs + ((16 * ct + 4 * cgl) * R + slot) * WR_KP + 16 * kxc + kxl;
#pragma unroll
            for (int c = 0; c < 4; ++c) dst[c * R * WR_KP] = (unsigned short)((c < 2 ? xr[u].x : xr[u].y) >> (16 * (c & 1)));
        }
        __syncthreads();
        if (sg + 1 < se) load_step();
#pragma unroll
        for (int qi = 0; qi < QI; ++qi) {
            const int item = wave + 4 * qi;
            const int tap = item % 9, ct = (item / 9) % NT, cm = item / (9 * NT);
            if (item >= NI || ct * 16 >= ncv) continue;  // uniform over the wave
            const int dyy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int j = 0; j < YB; ++j) {
                const int slot = (y0 + j + dyy) % R;  // input row y0 + j + dy - 1
                const uint4 av = *reinterpret_cast<const uint4*>(
                    Ps + (((dx * TM + cm) * 16 + (lane & 15)) * YB + j) * WR_KP + (lane >> 4) * 8);
                const uint4 bv = *reinterpret_cast<const uint4*>(
                    Xs + ((ct * 16 + (lane & 15)) * R + slot) * WR_KP + (lane >> 4) * 8);
                acc[qi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, av),
                                                                  __builtin_bit_cast(bf8v, bv), acc[qi], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D[i = co][j = ci]: lane holds co = 16 cm + 4 (l/16) + e, ci = c0 + 16 ct + l % 16
    float* P = part + (size_t)blockIdx.x * g.Cout * 27 * Cin;
#pragma unroll
    for (int qi = 0; qi < QI; ++qi) {
        const int item = wave + 4 * qi;
        const int tap = item % 9, ct = (item / 9) % NT, cm = item / (9 * NT);
        const int t = dz * 9 + tap;
        const int ci = c0 + ct * 16 + (lane & 15);
        if (item >= NI || ct * 16 >= ncv || ci >= Cin) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = cm * 16 + (lane >> 4) * 4 + e;
            if (co < g.Cout) P[((size_t)co * 27 + t) * Cin + ci] = acc[qi][e];
        }
    }
}

// channel groups of 4 per block of the row-segment kernel: whole 16-channel
// tiles, at most 64 channels
static int wgrad_rows_ng(const ConvGeom& g)
{
    const int c16 = ((g.Ca + g.Cb + 15) / 16) * 16;
    return c16 >= 64 ? 16 : c16 / 4;
}

// dW[q] = sum_c part[c][q], dW fp32.  A block takes 64 consecutive q; its 4
// waves sum the parts c = w, w + 4, ... (w = wave) with 8 loads in flight,
// then the 4 wave sums are added in wave order (a fixed order throughout).
__global__ void __launch_bounds__(256) reduce_parts_kernel(const float* __restrict__ part, int nparts, long long q_n,
                                                           float* __restrict__ out)
{
    __shared__ float red[4][64];
    const int l = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const long long q = (long long)blockIdx.x * 64 + l;
    float s = 0.f;
    if (q < q_n) {
        const float* src = part + q;
        int c = w;
        for (; c + 28 < nparts; c += 32) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = src[(size_t)(c + 4 * k) * q_n];
#pragma unroll
            for (int k = 0; k < 8; ++k) s += v[k];
        }
        for (; c < nparts; c += 4) s += src[(size_t)c * q_n];
    }
    red[w][l] = s;
    __syncthreads();
    if (w == 0 && q < q_n) out[q] = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
}

// bias gradient partials: part[chunk][co] = sum_{o in chunk} P[o][co], one
// pass over dL/dy: thread t takes channel group t % G (4 channels, one 16-byte
// load) of the voxels o = t / G, t / G + 256 / G, ... (G = Cout / 4), then
// the threads of a group are summed in a fixed tree order.
__global__ void __launch_bounds__(256) bias_grad_kernel(const float* __restrict__ dy, const unsigned short* __restrict__ y,
                                                        float slope, const unsigned short* __restrict__ pbf, long long M,
                                                        int Cout, long long VC, float* __restrict__ part)
{
    __shared__ float red[4][256];
    const int G = Cout / 4;                  // Cout is a multiple of 4, at most 1024
    const int T = (256 / G) * G;             // threads in use
    const int cg = (int)threadIdx.x % G, vs = (int)threadIdx.x / G, nv = 256 / G;
    const long long ob = (long long)blockIdx.x * VC, oe = min(M, ob + VC);
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    if ((int)threadIdx.x < T && pbf) {  // P given in bf16: 4 voxels' loads in flight, added in voxel order
        long long o = ob + vs;
        for (; o + 3 * nv < oe; o += 4 * nv) {
            s4v pv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) pv[k] = ld4bf(pbf + (size_t)(o + k * nv) * Cout + 4 * cg);
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < 4; ++c) s[c] += bf2f((unsigned short)pv[k][c]);
        }
        for (; o < oe; o += nv) {
            const s4v pv = ld4bf(pbf + (size_t)o * Cout + 4 * cg);
#pragma unroll
            for (int c = 0; c < 4; ++c) s[c] += bf2f((unsigned short)pv[c]);
        }
    } else if ((int)threadIdx.x < T) {
        for (long long o = ob + vs; o < oe; o += nv) {
            const size_t i = (size_t)o * Cout + 4 * cg;
            const float4 d = *reinterpret_cast<const float4*>(dy + i);
            const float pv[4] = {d.x, d.y, d.z, d.w};
            float f[4] = {1.f, 1.f, 1.f, 1.f};
            if (y) {
                const s4v yv = ld4bf(y + i);
#pragma unroll
                for (int c = 0; c < 4; ++c) f[c] = lrelu_d((unsigned short)yv[c], slope);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)  // the same bf16 operand the weight gradient uses
                s[c] += __uint_as_float((unsigned)f2bf(pv[c] * f[c]) << 16);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    // sum over the voxel slots vs of each group: slot stride G in the thread index
    for (int h = 1; h < nv; h <<= 1) {  // nv is a power of two (G divides 256 only then is T = 256)
        if (vs % (2 * h) == 0 && vs + h < nv && (int)threadIdx.x < T)
#pragma unroll
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + h * G];
        __syncthreads();
    }
    if (vs == 0 && (int)threadIdx.x < G)
#pragma unroll
        for (int c = 0; c < 4; ++c) part[(size_t)blockIdx.x * Cout + 4 * cg + c] = red[c][threadIdx.x];
}

// ------------------------------------------------------------ small kernels --
__global__ void __launch_bounds__(256) cast_bf16_kernel(const float* __restrict__ x, long long n,
                                                        unsigned short* __restrict__ y)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        y[i] = f2bf(x[i]);
}

// W [Cout][27][Cin] fp32 -> bf16 copy and bf16 transpose [Cin][27][Cout]
__global__ void __launch_bounds__(256) weight_prep_kernel(const float* __restrict__ w, int Cout, int Cin,
                                                          unsigned short* __restrict__ wbf,
                                                          unsigned short* __restrict__ wt)
{
    const int n = Cout * 27 * Cin;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const int co = i / (27 * Cin), r = i - co * 27 * Cin, t = r / Cin, ci = r - t * Cin;
        const unsigned short h = f2bf(w[i]);
        if (wbf) wbf[i] = h;
        if (wt) wt[((size_t)ci * 27 + t) * Cout + co] = h;
    }
}

// (F, M) fp32 [N][D][H][W] each -> bf16 [N][D][H][W][4] = (F, M, 0, 0)
__global__ void __launch_bounds__(256) pack_pair_kernel(const float* __restrict__ F, const float* __restrict__ M,
                                                        long long nvox, unsigned short* __restrict__ x)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < nvox; i += (long long)gridDim.x * 256) {
        uint2 v;
        v.x = (unsigned)f2bf(F[i]) | ((unsigned)f2bf(M[i]) << 16);
        v.y = 0u;
        *reinterpret_cast<uint2*>(x + 4 * i) = v;
    }
}

// split the gradient of a concatenated, upsampled input: dXcat fp32 [N][Di][Hi][Wi][Ca+Cb]
//   dxb[n,z,y,x,c]  (+)= dXcat[..., Ca + c]
//   dxa[n,Z,Y,X,c]  (+)= sum over the 8 fine voxels (2Z+a, 2Y+b, 2X+c) of dXcat[..., c]
// One block per coarse row (n, Z, Y): it writes dxa of that row and dxb of the
// 4 fine rows (2Z + a, 2Y + b) beneath it, so that the two parts of each
// fine voxel's channels are read by the same block at about the same time
// (a cache line holds both).  Work item (X, k): k < Ca/4 sums channel group k
// of the 8 fine voxels of coarse voxel X (in (a, b, c) order); k = Ca/4 +
// 8 f + q copies channel group q of the skip part of fine voxel f = 4a + 2b + c.
// 16-byte loads and stores (Ca and Cb are multiples of 4, the pointers
// 16-byte aligned).
__global__ void __launch_bounds__(256) split_grad_kernel(ConvGeom g, const float* __restrict__ dxc,
                                                         float* __restrict__ dxa, float* __restrict__ dxb, int acc_a,
                                                         int acc_b)
{
    const int Cin = g.Ca + g.Cb;
    const int R = (int)blockIdx.x;
    const int Da = g.Di >> 1, Ha = g.Hi >> 1, Wa = g.Wi >> 1;
    const int Y = R % Ha, Z = (R / Ha) % Da, n = R / (Ha * Da);
    const int Ga = g.Ca >> 2, Gb = g.Cb >> 2, K = Ga + 8 * Gb;
    const int XC = max(1, (1 << 24) / K);  // X positions per pass: 32-bit item indices
    for (int X0 = 0; X0 < Wa; X0 += XC) {
        const int nit = min(XC, Wa - X0) * K;
        for (int it = (int)threadIdx.x; it < nit; it += 256) {
            const int X = X0 + it / K, k = it % K;
            if (k < Ga) {
                float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c) {
                            const size_t f = (((size_t)n * g.Di + 2 * Z + a) * g.Hi + 2 * Y + b) * g.Wi + 2 * X + c;
                            const float4 v = *reinterpret_cast<const float4*>(dxc + f * Cin + 4 * k);
                            s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
                        }
                float4* d = reinterpret_cast<float4*>(dxa + ((size_t)R * Wa + X) * g.Ca + 4 * k);
                if (acc_a) {
                    const float4 o = *d;
                    s = make_float4(o.x + s.x, o.y + s.y, o.z + s.z, o.w + s.w);
                }
                *d = s;
            } else {
                const int kk = k - Ga, fv = kk / Gb, q = kk - fv * Gb;
                const int a = fv >> 2, b = (fv >> 1) & 1, c = fv & 1;
                const size_t f = (((size_t)n * g.Di + 2 * Z + a) * g.Hi + 2 * Y + b) * g.Wi + 2 * X + c;
                const float4 s = *reinterpret_cast<const float4*>(dxc + f * Cin + g.Ca + 4 * q);
                float4* d = reinterpret_cast<float4*>(dxb + f * g.Cb + 4 * q);
                if (acc_b) {
                    const float4 o = *d;
                    *d = make_float4(o.x + s.x, o.y + s.y, o.z + s.z, o.w + s.w);
                } else {
                    *d = s;
                }
            }
        }
    }
}

// MSE between pred [N][D][H][W][Cp] channels 0..2 and target [N][3][D][H][W]:
// grad (written to dpred, channels >= 3 zeroed) and per-block partial sums.
__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ pred, int Cp,
                                                  const float* __restrict__ tgt, long long nvox_per, int N,
                                                  float* __restrict__ dpred, double* __restrict__ part, double scale)
{
    __shared__ double red[256];
    double s = 0.0;
    const long long nv = nvox_per * N;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < nv; i += (long long)gridDim.x * 256) {
        const long long n = i / nvox_per, v = i - n * nvox_per;
        for (int c = 0; c < Cp; ++c) {
            float g = 0.f;
            if (c < 3) {
                const float d = pred[i * Cp + c] - tgt[(n * 3 + c) * nvox_per + v];
                s += (double)d * d;
                g = (float)(2.0 * scale) * d;
            }
            if (dpred) dpred[i * Cp + c] = g;
        }
    }
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s * scale;
}

// *out = sum of the partials (fixed order)
__global__ void __launch_bounds__(256) sum_partials_kernel(const double* __restrict__ part, int n, float* out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) *out = (float)s;
}

// pred [N][D][H][W][Cp] -> displacement [N][3][D][H][W]
__global__ void __launch_bounds__(256) unpack_disp_kernel(const float* __restrict__ pred, int Cp, long long nvox_per,
                                                          int N, float* __restrict__ u)
{
    const long long nv = nvox_per * N;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < nv; i += (long long)gridDim.x * 256) {
        const long long n = i / nvox_per, v = i - n * nvox_per;
        for (int c = 0; c < 3; ++c) u[(n * 3 + c) * nvox_per + v] = pred[i * Cp + c];
    }
}

// ------------------------------------------------------------------ host ----
static unsigned grid_for(long long n, int per = 256, long long cap = 16384)
{
    long long b = (n + per - 1) / per;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <bool C8>
static void launch_fwd(int nt, unsigned blocks, hipStream_t st, const ConvGeom& g, const unsigned short* xa,
                       const unsigned short* xb, const unsigned short* w, const float* bias, int act, float slope,
                       unsigned short* ybf, float* yf)
{
    // up to 2 output-channel tiles: 2 voxel tiles per wave (a block covers 128
    // voxels); with 4 or 8 the kernel is faster with one (fewer registers)
    const unsigned b2 = (blocks + 1) / 2;
    if (nt <= 1) hipLaunchKernelGGL((conv_fwd_kernel<1, C8, 2>), dim3(b2), dim3(256), 0, st, g, xa, xb, w, bias, act, slope, ybf, yf);
    else if (nt <= 2) hipLaunchKernelGGL((conv_fwd_kernel<2, C8, 2>), dim3(b2), dim3(256), 0, st, g, xa, xb, w, bias, act, slope, ybf, yf);
    else if (nt <= 4) hipLaunchKernelGGL((conv_fwd_kernel<4, C8, 1>), dim3(blocks), dim3(256), 0, st, g, xa, xb, w, bias, act, slope, ybf, yf);
    else hipLaunchKernelGGL((conv_fwd_kernel<8, C8, 1>), dim3(blocks), dim3(256), 0, st, g, xa, xb, w, bias, act, slope, ybf, yf);
}

hipError_t conv_fwd_launch(const ConvGeom& g, const unsigned short* xa, const unsigned short* xb,
                           const unsigned short* w, const float* bias, int act, float slope, unsigned short* ybf,
                           float* yf, hipStream_t st)
{
    const long long M = (long long)g.N * g.Do * g.Ho * g.Wo;
    const unsigned blocks = (unsigned)((M + 63) / 64);
    const int nt = (g.Cout + 15) / 16;
    if (nt > 8) return hipErrorInvalidValue;
    if (g.Ca % 8 == 0 && g.Cb % 8 == 0) launch_fwd<true>(nt, blocks, st, g, xa, xb, w, bias, act, slope, ybf, yf);
    else launch_fwd<false>(nt, blocks, st, g, xa, xb, w, bias, act, slope, ybf, yf);
    return hipGetLastError();
}

template <bool C8, bool PAR, bool PB, int MT>
static void launch_bwd_data(int nt, unsigned blocks, hipStream_t st, const ConvGeom& g, const float* dy,
                            const unsigned short* y, float slope, const unsigned short* pb, const unsigned short* wt,
                            float* dx, int accumulate)
{
#define BWD_DATA(T) \
    hipLaunchKernelGGL((conv_bwd_data_kernel<T, C8, PAR, PB, MT>), dim3(blocks), dim3(256), 0, st, g, dy, y, slope, pb, wt, dx, accumulate)
    if constexpr (MT == 2) {  // nt <= 3
        if (nt <= 1) BWD_DATA(1);
        else if (nt <= 2) BWD_DATA(2);
        else BWD_DATA(3);
    } else {  // nt >= 4
        if (nt <= 4) BWD_DATA(4);
        else if (nt <= 6) BWD_DATA(6);
        else if (nt <= 8) BWD_DATA(8);
        else BWD_DATA(12);
    }
#undef BWD_DATA
}

template <bool PB>
static hipError_t bwd_data_dispatch(const ConvGeom& g, const float* dy, const unsigned short* y, float slope,
                                    const unsigned short* pb, const unsigned short* wt, float* dx, int accumulate,
                                    hipStream_t st)
{
    const int nt = (g.Ca + g.Cb + 15) / 16;
    if (nt > 12) return hipErrorInvalidValue;
    // up to 3 input-channel tiles: 2 voxel tiles per wave, so that each LDS
    // read of the weights feeds two MFMAs (a block covers 128 voxels)
    const int MTv = nt <= 3 ? 2 : 1;
    if (g.stride == 2) {  // 8 parity classes of the half-resolution grid (rounded up)
        const long long Mc = (long long)g.N * ((g.Di + 1) / 2) * ((g.Hi + 1) / 2) * ((g.Wi + 1) / 2);
        const unsigned blocks = (unsigned)(8 * ((Mc + 64 * MTv - 1) / (64 * MTv)));
        if (MTv == 2) {
            if (g.Cout % 8 == 0) launch_bwd_data<true, true, PB, 2>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
            else launch_bwd_data<false, true, PB, 2>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
        } else {
            if (g.Cout % 8 == 0) launch_bwd_data<true, true, PB, 1>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
            else launch_bwd_data<false, true, PB, 1>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
        }
    } else {
        const long long M = (long long)g.N * g.Di * g.Hi * g.Wi;
        const unsigned blocks = (unsigned)((M + 64 * MTv - 1) / (64 * MTv));
        if (MTv == 2) {
            if (g.Cout % 8 == 0) launch_bwd_data<true, false, PB, 2>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
            else launch_bwd_data<false, false, PB, 2>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
        } else {
            if (g.Cout % 8 == 0) launch_bwd_data<true, false, PB, 1>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
            else launch_bwd_data<false, false, PB, 1>(nt, blocks, st, g, dy, y, slope, pb, wt, dx, accumulate);
        }
    }
    return hipGetLastError();
}

hipError_t conv_bwd_data_launch(const ConvGeom& g, const float* dy, const unsigned short* y, float slope,
                                const unsigned short* wt, float* dx, int accumulate, hipStream_t st)
{
    return bwd_data_dispatch<false>(g, dy, y, slope, nullptr, wt, dx, accumulate, st);
}

hipError_t conv_bwd_data_p_launch(const ConvGeom& g, const unsigned short* p, const unsigned short* wt, float* dx,
                                  int accumulate, hipStream_t st)
{
    return bwd_data_dispatch<true>(g, nullptr, nullptr, 0.0f, p, wt, dx, accumulate, st);
}

// P = bf16(dL/dy act'(y)) elementwise (y NULL: the identity), the rounding of
// the operand packing in the backward kernels (round to nearest even).
__global__ void __launch_bounds__(256) act_grad_kernel(const float* __restrict__ dy, const unsigned short* __restrict__ y,
                                                       float slope, long long n, unsigned short* __restrict__ p)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        float v = dy[i];
        if (y) v *= lrelu_d(y[i], slope);
        p[i] = f2bf(v);
    }
}

// The same, 8 elements per thread and step (n8 groups of 8; 16-byte aligned
// operands): two 16-byte loads of dy, one of y, one 16-byte store.
__global__ void __launch_bounds__(256) act_grad8_kernel(const float* __restrict__ dy,
                                                        const unsigned short* __restrict__ y, float slope, long long n8,
                                                        unsigned short* __restrict__ p)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n8; i += (long long)gridDim.x * 256) {
        const float4 d0 = reinterpret_cast<const float4*>(dy)[2 * i];
        const float4 d1 = reinterpret_cast<const float4*>(dy)[2 * i + 1];
        float v[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
        if (y) {
            const uint4 yv = reinterpret_cast<const uint4*>(y)[i];
            const unsigned yw[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] *= lrelu_d((unsigned short)(yw[q >> 1] >> (16 * (q & 1))), slope);
        }
        uint4 o;
        o.x = (unsigned)f2bf(v[0]) | ((unsigned)f2bf(v[1]) << 16);
        o.y = (unsigned)f2bf(v[2]) | ((unsigned)f2bf(v[3]) << 16);
        o.z = (unsigned)f2bf(v[4]) | ((unsigned)f2bf(v[5]) << 16);
        o.w = (unsigned)f2bf(v[6]) | ((unsigned)f2bf(v[7]) << 16);
        reinterpret_cast<uint4*>(p)[i] = o;
    }
}

hipError_t act_grad_launch(const float* dy, const unsigned short* y, float slope, long long n, unsigned short* p,
                           hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const bool a16 = ((reinterpret_cast<uintptr_t>(dy) | reinterpret_cast<uintptr_t>(y) |
                       reinterpret_cast<uintptr_t>(p)) & 15u) == 0;
    long long head = 0;  // elements done by the vector kernel
    if (a16 && n >= 8) {
        const long long n8 = n / 8;
        long long blocks = (n8 + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(act_grad8_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dy, y, slope, n8, p);
        head = n8 * 8;
    }
    if (head < n) {
        const long long rest = n - head;
        long long blocks = (rest + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(act_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dy + head, y ? y + head : nullptr,
                           slope, rest, p + head);
    }
    return hipGetLastError();
}

// Row pitch of P^T: the output voxels rounded up to 8.
static long long wgrad_mp(long long M) { return (M + 7) / 8 * 8; }

// The all-taps kernel for layers with at most 3 tiles of 16 x 16 (co, ci).
static bool wgrad_all_taps(const ConvGeom& g)
{
    const int tm = (g.Cout + 15) / 16, tn = (g.Ca + g.Cb + 15) / 16;
    return tm * tn <= 3;
}

static bool wgrad_rows(const ConvGeom& g) { return g.stride == 1 && g.Cout <= 64; }

ConvWgradPlan conv_wgrad_plan(const ConvGeom& g)
{
    ConvWgradPlan p;
    const long long M = (long long)g.N * g.Do * g.Ho * g.Wo;
    p.rows = 0;
    p.VS = 0;
    if (wgrad_rows(g)) {
        // about 2048 blocks over (chunk, dz, channel chunk)
        const int yb = wgrad_rows_yb((g.Cout + 15) / 16);
        const long long S = (long long)g.N * g.Do * ((g.Ho + yb - 1) / yb) * ((g.Wo + WR_SEG - 1) / WR_SEG);
        const int ncc = (g.Ca + g.Cb + 4 * wgrad_rows_ng(g) - 1) / (4 * wgrad_rows_ng(g));
        long long want = (2048 + 3 * ncc - 1) / (3 * ncc);
        if (want > S) want = S;
        p.rows = 1;
        p.VS = (S + want - 1) / want;
        p.nchunks = (int)((S + p.VS - 1) / p.VS);
        p.VC = (M + p.nchunks - 1) / p.nchunks;  // bias partials: the same number of chunks
        const long long q = (long long)g.Cout * 27 * (g.Ca + g.Cb);
        p.part_floats = (long long)p.nchunks * q + (long long)p.nchunks * g.Cout;
        return p;
    }
    // all-taps kernel: about 1024 chunks (each block covers every tap);
    // tap-per-block kernel: about 256 chunks x 27 taps
    long long vc = (M + (wgrad_all_taps(g) ? 1023 : 255)) / (wgrad_all_taps(g) ? 1024 : 256);
    vc = ((vc + 31) / 32) * 32;
    if (vc < 256) vc = 256;
    p.VC = vc;
    p.nchunks = (int)((M + vc - 1) / vc);
    const long long q = (long long)g.Cout * 27 * (g.Ca + g.Cb);
    // partials, bias partials, then P^T (bf16 [Cout][MP], 16-byte aligned)
    p.part_floats = (long long)p.nchunks * q + (long long)p.nchunks * g.Cout + (g.Cout * wgrad_mp(M) + 1) / 2 + 4;
    return p;
}

template <int TM>
static void launch_wg_tm(int tnw, dim3 grid, hipStream_t st, const ConvGeom& g, const unsigned short* xa,
                         const unsigned short* xb, const unsigned short* pt, long long MP, long long VC, float* part)
{
    if (tnw <= 1) hipLaunchKernelGGL((conv_bwd_weight_kernel<TM, 1>), grid, dim3(256), 0, st, g, xa, xb, pt, MP, VC, part);
    else if (tnw <= 2) hipLaunchKernelGGL((conv_bwd_weight_kernel<TM, 2>), grid, dim3(256), 0, st, g, xa, xb, pt, MP, VC, part);
    else hipLaunchKernelGGL((conv_bwd_weight_kernel<TM, 3>), grid, dim3(256), 0, st, g, xa, xb, pt, MP, VC, part);
}

template <int TM, bool PB>
static void launch_wgrad_rows_tm(int ng, dim3 grid, hipStream_t st, const ConvGeom& g, const unsigned short* xa,
                                 const unsigned short* xb, const float* dy, const unsigned short* y, float slope,
                                 const unsigned short* pbf, long long VS, float* part)
{
    if (ng == 4) hipLaunchKernelGGL((conv_wgrad_rows_kernel<TM, 4, PB>), grid, dim3(256), 0, st, g, xa, xb, dy, y, slope, pbf, VS, part);
    else if (ng == 8) hipLaunchKernelGGL((conv_wgrad_rows_kernel<TM, 8, PB>), grid, dim3(256), 0, st, g, xa, xb, dy, y, slope, pbf, VS, part);
    else if (ng == 12) hipLaunchKernelGGL((conv_wgrad_rows_kernel<TM, 12, PB>), grid, dim3(256), 0, st, g, xa, xb, dy, y, slope, pbf, VS, part);
    else hipLaunchKernelGGL((conv_wgrad_rows_kernel<TM, 16, PB>), grid, dim3(256), 0, st, g, xa, xb, dy, y, slope, pbf, VS, part);
}

template <bool PB>
static void launch_wgrad_rows(int tm, int ng, dim3 grid, hipStream_t st, const ConvGeom& g, const unsigned short* xa,
                              const unsigned short* xb, const float* dy, const unsigned short* y, float slope,
                              const unsigned short* pbf, long long VS, float* part)
{
    if (tm == 1) launch_wgrad_rows_tm<1, PB>(ng, grid, st, g, xa, xb, dy, y, slope, pbf, VS, part);
    else if (tm == 2) launch_wgrad_rows_tm<2, PB>(ng, grid, st, g, xa, xb, dy, y, slope, pbf, VS, part);
    else launch_wgrad_rows_tm<4, PB>(ng, grid, st, g, xa, xb, dy, y, slope, pbf, VS, part);
}

// P = dL/dy act'(y) from dy and y, or given in bf16 (pbf non-NULL)
static hipError_t bwd_weight_run(const ConvGeom& g, const unsigned short* xa, const unsigned short* xb,
                                 const float* dy, const unsigned short* y, float slope, const unsigned short* pbf,
                                 float* dw, float* db, float* part, hipStream_t st)
{
    const ConvWgradPlan p = conv_wgrad_plan(g);
    const int Cin = g.Ca + g.Cb;
    const int tm = (g.Cout + 15) / 16, tn = (Cin + 15) / 16, tnw = (tn + 3) / 4;
    if (tnw > 3 || tm > 8) return hipErrorInvalidValue;
    if (p.rows) {
        const int ng = wgrad_rows_ng(g);
        dim3 grid(p.nchunks, 3 * ((Cin + 4 * ng - 1) / (4 * ng)));
        if (pbf) launch_wgrad_rows<true>(tm, ng, grid, st, g, xa, xb, dy, y, slope, pbf, p.VS, part);
        else launch_wgrad_rows<false>(tm, ng, grid, st, g, xa, xb, dy, y, slope, pbf, p.VS, part);
    } else {
        // P^T first (the voxel-chunk kernels read their A operands from it)
        const long long M = (long long)g.N * g.Do * g.Ho * g.Wo, MP = wgrad_mp(M);
        const uintptr_t pa = reinterpret_cast<uintptr_t>(part + (size_t)p.nchunks * (g.Cout * 27LL * Cin + g.Cout));
        unsigned short* pt = reinterpret_cast<unsigned short*>((pa + 15) & ~(uintptr_t)15);
        hipLaunchKernelGGL(p_transpose_kernel, dim3((unsigned)((MP + 63) / 64)), dim3(256), 0, st, dy, y, slope, pbf,
                           M, g.Cout, MP, pt);
        if (wgrad_all_taps(g)) {
            dim3 grid1(p.nchunks);
            if (tm == 1 && tn == 1) hipLaunchKernelGGL((conv_bwd_weight_taps_kernel<1, 1>), grid1, dim3(256), 0, st, g, xa, xb, pt, MP, p.VC, part);
            else if (tm == 1 && tn == 2) hipLaunchKernelGGL((conv_bwd_weight_taps_kernel<1, 2>), grid1, dim3(256), 0, st, g, xa, xb, pt, MP, p.VC, part);
            else if (tm == 1) hipLaunchKernelGGL((conv_bwd_weight_taps_kernel<1, 3>), grid1, dim3(256), 0, st, g, xa, xb, pt, MP, p.VC, part);
            else if (tm == 2) hipLaunchKernelGGL((conv_bwd_weight_taps_kernel<2, 1>), grid1, dim3(256), 0, st, g, xa, xb, pt, MP, p.VC, part);
            else hipLaunchKernelGGL((conv_bwd_weight_taps_kernel<3, 1>), grid1, dim3(256), 0, st, g, xa, xb, pt, MP, p.VC, part);
        } else {
            dim3 grid(p.nchunks, 27);
            switch (tm) {
                case 1: launch_wg_tm<1>(tnw, grid, st, g, xa, xb, pt, MP, p.VC, part); break;
                case 2: launch_wg_tm<2>(tnw, grid, st, g, xa, xb, pt, MP, p.VC, part); break;
                case 3: case 4: launch_wg_tm<4>(tnw, grid, st, g, xa, xb, pt, MP, p.VC, part); break;
                default: launch_wg_tm<8>(tnw, grid, st, g, xa, xb, pt, MP, p.VC, part); break;
            }
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long q = (long long)g.Cout * 27 * Cin;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((q + 63) / 64)), dim3(256), 0, st, part, p.nchunks, q, dw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (db) {
        const long long M = (long long)g.N * g.Do * g.Ho * g.Wo;
        float* pb = part + (size_t)p.nchunks * q;
        hipLaunchKernelGGL(bias_grad_kernel, dim3(p.nchunks), dim3(256), 0, st, dy, y, slope, pbf, M, g.Cout, p.VC,
                           pb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)((g.Cout + 63) / 64)), dim3(256), 0, st, pb, p.nchunks,
                           (long long)g.Cout, db);
        e = hipGetLastError();
    }
    return e;
}

hipError_t conv_bwd_weight_launch(const ConvGeom& g, const unsigned short* xa, const unsigned short* xb,
                                  const float* dy, const unsigned short* y, float slope, float* dw, float* db,
                                  float* part, hipStream_t st)
{
    return bwd_weight_run(g, xa, xb, dy, y, slope, nullptr, dw, db, part, st);
}

hipError_t conv_bwd_weight_p_launch(const ConvGeom& g, const unsigned short* xa, const unsigned short* xb,
                                    const unsigned short* p, float* dw, float* db, float* part, hipStream_t st)
{
    return bwd_weight_run(g, xa, xb, nullptr, nullptr, 0.0f, p, dw, db, part, st);
}

hipError_t cast_bf16_launch(const float* x, long long n, unsigned short* y, hipStream_t st)
{
    hipLaunchKernelGGL(cast_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, n, y);
    return hipGetLastError();
}

hipError_t weight_prep_launch(const float* w, int Cout, int Cin, unsigned short* wbf, unsigned short* wt,
                              hipStream_t st)
{
    hipLaunchKernelGGL(weight_prep_kernel, dim3(grid_for((long long)Cout * 27 * Cin)), dim3(256), 0, st, w, Cout, Cin,
                       wbf, wt);
    return hipGetLastError();
}

hipError_t pack_pair_launch(const float* F, const float* M, long long nvox, unsigned short* x, hipStream_t st)
{
    hipLaunchKernelGGL(pack_pair_kernel, dim3(grid_for(nvox)), dim3(256), 0, st, F, M, nvox, x);
    return hipGetLastError();
}

hipError_t split_grad_launch(const ConvGeom& g, const float* dxc, float* dxa, float* dxb, int acc_a, int acc_b,
                             hipStream_t st)
{
    const int Rc = g.N * (g.Di >> 1) * (g.Hi >> 1);  // coarse rows: the voxel count is below 2^31
    hipLaunchKernelGGL(split_grad_kernel, dim3((unsigned)Rc), dim3(256), 0, st, g, dxc, dxa, dxb, acc_a, acc_b);
    return hipGetLastError();
}

hipError_t mse_launch(const float* pred, int Cp, const float* tgt, long long nvox_per, int N, float* dpred,
                      double* part, int nblocks, float* loss, hipStream_t st)
{
    const double scale = 1.0 / ((double)nvox_per * N * 3.0);
    hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, st, pred, Cp, tgt, nvox_per, N, dpred, part, scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (loss) {
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, part, nblocks, loss);
        e = hipGetLastError();
    }
    return e;
}

hipError_t unpack_disp_launch(const float* pred, int Cp, long long nvox_per, int N, float* u, hipStream_t st)
{
    hipLaunchKernelGGL(unpack_disp_kernel, dim3(grid_for(nvox_per * N)), dim3(256), 0, st, pred, Cp, nvox_per, N, u);
    return hipGetLastError();
}

}  // namespace ffdp
