// Fused warp + LNCC forward and adjoint for gfx950.
//
// What is computed (App. "Definition of LNCC loss", Alg. fusedlncc):
//   Mw(x) = M(x + u(x))                         trilinear, never stored
//   mu_F, mu_M, mu_FF, mu_MM, mu_FM             w^3 box means, zero padding
//   A = mu_FM - mu_F mu_M, B = mu_FF - mu_F^2, C = mu_MM - mu_M^2
//   n_i = A^2 / (B C + eps);  loss = 1 - mean_{ROI} n_i
// and, for the adjoint to the moving image (eq. finalccgradM, redone for the
// warped image with eps kept and g_i = dL/dn_i = -1/N_roi on the ROI):
//   a_i = 2 g_i A_i / D_i,  c_i = a_i A_i B_i / D_i,  e_i = c_i mu_M,i - a_i mu_F,i
//   dL/dMw_k = F_k (w*a)_k - Mw_k (w*c)_k + (w*e)_k        (D_i = B_i C_i + eps)
//   dL/du_k  = dL/dMw_k * dMw_k/dp                          (Alg. gridsampler Backward)
// The paper keeps five gamma fields for F and M; only the moving image is
// differentiated here, so three fields (a, c, e) suffice.
//
// Design (one kernel, nothing N-sized in HBM besides inputs and grad_u):
//  * a block of 512 threads owns a 32 x 16 column tile and a z-chunk and
//    streams z slices through a pipeline of LDS stages (the w = 7 adjoint:
//    768 threads and 32 x 24 tiles, see lncc_tile);
//  * stage A samples F and Mw on the tile plus a halo of 2r (r for the
//    forward) and keeps the last w slices of every column in registers; for
//    the tile's own voxel (one per thread) it also keeps dMw/dp in a
//    thread-private LDS ring, so the output stage never samples again.  It
//    writes the five z-window sums to LDS;
//  * loads are software-pipelined over slices: the eight M corners, the
//    cell fractions and F of slice z+1 are fetched while slice z goes
//    through stages B-F, so stage A only interpolates;
//  * stage B sums x-windows, stage C y-windows, forms A, B, C, the loss term
//    and a, c, e; stage D boxes a, c, e in x; stage E boxes them in y and
//    scatters F(zo) a - Mw(zo) c + e into the accumulators of the 2r+1
//    pending output slices of the thread's column (the z-window), and the
//    oldest one becomes grad_u with dMw/dp from the ring;
//  * the x- and y-window passes read and write 2 floats per LDS access;
//  * statistics use values shifted by a per-block constant (F and M at the
//    tile centre).  With padded voxels shifted too, A, B, C and the adjoint
//    are unchanged in exact arithmetic and the fp32 cancellation in
//    B = mu_FF - mu_F^2 shrinks;
//  * window sums are direct w-term sums (no running add/subtract drift).
#include "device.hpp"
#include "internal.hpp"

namespace ffdp {

enum { MODE_FWD = 0, MODE_BWD = 1, MODE_ANTS = 2 };

__host__ __device__ constexpr int round4(int v) { return (v + 3) & ~3; }

template <int WIN, int MODE, int TX_, int TY_>
struct LnccTile {
    static constexpr int r = (WIN - 1) / 2;
    static constexpr int TX = TX_, TY = TY_, NT = TX_ * TY_;
    static constexpr int R2 = (MODE == MODE_BWD) ? 2 * r : r;  // stage-A halo
    static constexpr int R1 = (MODE == MODE_BWD) ? r : 0;      // stage-C halo
    static constexpr int X2 = TX + 2 * R2, Y2 = TY + 2 * R2;
    static constexpr int X1 = TX + 2 * R1, Y1 = TY + 2 * R1;
    // One LDS row pitch for stage-A data and its x-windowed copy, so that the
    // 2-wide runs of stages B and C map consecutive lanes to consecutive
    // addresses (no bank conflicts where a wave crosses rows).  Runs past X1
    // read the next row and produce values that are never used.
    static constexpr int X2p = round4(X2 > X1 + 2 * r ? X2 : X1 + 2 * r);
    static constexpr int X1p = X2p;
    static constexpr int NV = (WIN + 2) / 2;         // float2 reads per 2-wide x-window run
    static constexpr int NA = Y2 * X2p;              // floats per channel, stage A
    static constexpr int NB = Y2 * X1p;              // x-window
    static constexpr int NC = Y1 * X1p;              // a, c, e
    static constexpr int ND = Y1 * TX;               // x-window of a, c, e
    static constexpr int NH = X2 * Y2 - TX * TY;     // halo-only stage-A points
    static constexpr int PH = (NH + NT - 1) / NT;
    static constexpr int NW = NT / 64;               // waves per block
    static constexpr int QW = (NH + NW - 1) / NW;    // halo points per wave when PH == 1
    static constexpr int RB = Y2 * X1p / 2;          // 2-wide runs, stage B
    static constexpr int RC = Y1 * X1p / 2;          // 2-wide runs, stage C (adjoint mode)
    static constexpr int RD = Y1 * TX / 2;           // 2-wide runs, stage D
    static constexpr int NG = (MODE != MODE_FWD) ? 3 * WIN * NT : 0;  // dMw/dp ring, thread-private
    // adjoint: the loss accumulator (one double per thread) also lives in LDS
    static constexpr int NL = (MODE == MODE_BWD) ? 2 * NT : 0;
    // LDS layout: the thread-private ring first, so that every slot is an
    // immediate offset (below 64 KB) from the thread's own address; then the
    // stage buffers and the loss doubles.
    static constexpr int OG = 0;
    static constexpr int OA = OG + NG;                  // stage A  [5][Y2][X2p]
    static constexpr int OB = OA + 5 * NA;              // stage B  [5][Y2][X1p]
    static constexpr int OL = (OB + 5 * NB + 1) & ~1;   // loss doubles
    static constexpr int LDS_FLOATS = OL + NL;
    static_assert(NT % 64 == 0 && TX % 2 == 0, "whole waves, 2-wide runs");
    static_assert(LDS_FLOATS * 4 <= 160 * 1024, "LDS of one CU");
    static_assert(3 * NC <= 5 * NA && 3 * ND <= 5 * NB, "aliased LDS buffers must fit");
};

// 2-wide run of w-tap window sums along a row: out[e] = sum_{d<w} row[e + d]
template <int WIN, int NV>
__device__ __forceinline__ float2 xwin2(const float* row)
{
    float v[2 * NV];
    const float2* src = reinterpret_cast<const float2*>(row);
#pragma unroll
    for (int n = 0; n < NV; ++n) {
        const float2 t = src[n];
        v[2 * n] = t.x;
        v[2 * n + 1] = t.y;
    }
    float o0 = v[0], o1 = v[1];
#pragma unroll
    for (int d = 1; d < WIN; ++d) {
        o0 += v[d];
        o1 += v[d + 1];
    }
    return make_float2(o0, o1);
}

// Addressing.  LNCC_ADDR32: the whole volume lies within 4 GB of its base, so
// loads and stores take 32-bit byte offsets from an SGPR base (one VALU add
// per address) and index products use the full-rate 24-bit multiplier.
// LNCC_ADDRWIN (volumes of 2^30 voxels or more, e.g. 1040^3): the same 32-bit
// form from per-block bases moved to slice zb, the first slice of a window of
// zspan slices that covers every slice the block streams; gathers whose
// corner slices fall outside the window (displacements of hundreds of slices)
// take 64-bit addresses, decided per wave.  LNCC_ADDR64: 64-bit element
// offsets throughout (shapes whose slices are too large for a window).
template <int ADDR>
__device__ __forceinline__ float ld(const float* __restrict__ base, unsigned idx)
{
    if (ADDR == LNCC_ADDR64) return base[idx];
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + idx * 4u);
}

// Element-index product.  The launcher selects the 32-bit forms only where
// every factor fits 24 bits (D, H*W < 2^24), so the full-rate 24-bit
// multiplier replaces the quarter-rate 32-bit one.
template <int ADDR>
__device__ __forceinline__ unsigned imul(int a, int b)
{
    if (ADDR == LNCC_ADDR64) return (unsigned)(a * b);
    return __umul24((unsigned)a, (unsigned)b);
}

// Two consecutive floats at element offset idx (4-byte aligned: one 8-byte load)
typedef float lncc_f2a __attribute__((ext_vector_type(2), aligned(4)));
template <int ADDR>
__device__ __forceinline__ lncc_f2a ld2(const float* __restrict__ base, unsigned idx)
{
    if (ADDR == LNCC_ADDR64) return *reinterpret_cast<const lncc_f2a*>(base + idx);
    return *reinterpret_cast<const lncc_f2a*>(reinterpret_cast<const char*>(base) + idx * 4u);
}

// grad_u is written once and not read again here: non-temporal stores
template <int ADDR>
__device__ __forceinline__ void st(float* __restrict__ base, unsigned idx, float v)
{
    if (ADDR == LNCC_ADDR64) __builtin_nontemporal_store(v, base + idx);
    else __builtin_nontemporal_store(v, reinterpret_cast<float*>(reinterpret_cast<char*>(base) + idx * 4u));
}

// Loads of one stage-A point for one slice, issued a slice ahead of their use.
// Border padding: the eight clamped M corners of the trilinear cell, the cell
// fractions and the derivative flags (sample point exactly on index 0 of an
// axis), plus F.  Zero padding: u and F only (the corners are fetched with
// their validity masks when the slice is consumed).
struct Pend {
    float c[8];
    float ax, ay, az;
    unsigned fl;
    float f;
};

// Mb and Fb are the (windowed) bases, M the volume itself; zb the window's
// first slice and zspan its length (ADDRWIN).  fidx is F's offset from Fb.
template <int PAD, int ADDR>
__device__ __forceinline__ void issue_point(Pend& g, const float* __restrict__ M, const float* __restrict__ Mb,
                                            const float* __restrict__ Fb, int D, int H, int W, int HW, int zb,
                                            int zspan, int x, int y, int z, unsigned fidx, float ux, float uy,
                                            float uz)
{
    g.f = ld<ADDR>(Fb, fidx);
    if (PAD != PAD_BORDER) {
        g.c[0] = ux; g.c[1] = uy; g.c[2] = uz;
        return;
    }
    const float fx = fminf(fmaxf(floorf(ux), -268435456.0f), 268435456.0f);
    const float fy = fminf(fmaxf(floorf(uy), -268435456.0f), 268435456.0f);
    const float fz = fminf(fmaxf(floorf(uz), -268435456.0f), 268435456.0f);
    const float ax = ux - fx;
    g.ay = uy - fy; g.az = uz - fz;
    const int ix = x + (int)fx, iy = y + (int)fy, iz = z + (int)fz;
    const int y0 = min(max(iy, 0), H - 1), y1 = min(max(iy + 1, 0), H - 1);
    const int z0 = min(max(iz, 0), D - 1), z1 = min(max(iz + 1, 0), D - 1);
    const unsigned p0 = imul<ADDR>(y0, W), p1 = imul<ADDR>(y1, W);
    if (ADDR == LNCC_ADDR64) {  // also every width-1 volume: one float per corner
        const int x0 = min(max(ix, 0), W - 1), x1 = min(max(ix + 1, 0), W - 1);
        const size_t q0 = (size_t)z0 * (size_t)HW, q1 = (size_t)z1 * (size_t)HW;
        g.ax = ax;
        g.c[0] = M[q0 + p0 + x0]; g.c[1] = M[q0 + p0 + x1];
        g.c[2] = M[q0 + p1 + x0]; g.c[3] = M[q0 + p1 + x1];
        g.c[4] = M[q1 + p0 + x0]; g.c[5] = M[q1 + p0 + x1];
        g.c[6] = M[q1 + p1 + x0]; g.c[7] = M[q1 + p1 + x1];
        g.fl = ((ix == 0 && ax == 0.0f) ? 1u : 0u) | ((iy == 0 && g.ay == 0.0f) ? 2u : 0u) |
               ((iz == 0 && g.az == 0.0f) ? 4u : 0u);
        return;
    }
    // x corners: one 8-byte load of columns xp, xp + 1 (the planner takes
    // these forms only for W >= 2).  A point clamped at the low border takes
    // the first of the pair (weight 0), at the high border the second
    // (weight 1, equal to it up to one rounding); either way its x
    // derivative is zero (flag bit 0).
    const bool xlo = ix < 0, xhi = ix >= W - 1;
    const int xp = min(max(ix, 0), W - 2);
    g.ax = xlo ? 0.0f : (xhi ? 1.0f : ax);
    bool fast = true;
    if (ADDR == LNCC_ADDRWIN)  // both corner slices inside the window, for every lane of the wave
        fast = __builtin_amdgcn_ballot_w64(!((unsigned)(z0 - zb) < (unsigned)zspan &&
                                             (unsigned)(z1 - zb) < (unsigned)zspan)) == 0;
    lncc_f2a v00, v01, v10, v11;
    if (ADDR != LNCC_ADDRWIN || fast) {
        const unsigned q0 = imul<ADDR>(z0 - zb, HW), q1 = imul<ADDR>(z1 - zb, HW);
        v00 = ld2<ADDR>(Mb, q0 + p0 + xp); v01 = ld2<ADDR>(Mb, q0 + p1 + xp);
        v10 = ld2<ADDR>(Mb, q1 + p0 + xp); v11 = ld2<ADDR>(Mb, q1 + p1 + xp);
    } else {  // a corner slice outside the window: 64-bit offsets
        const size_t q0 = (size_t)z0 * (size_t)HW, q1 = (size_t)z1 * (size_t)HW;
        v00 = *reinterpret_cast<const lncc_f2a*>(M + (q0 + p0 + xp));
        v01 = *reinterpret_cast<const lncc_f2a*>(M + (q0 + p1 + xp));
        v10 = *reinterpret_cast<const lncc_f2a*>(M + (q1 + p0 + xp));
        v11 = *reinterpret_cast<const lncc_f2a*>(M + (q1 + p1 + xp));
    }
    g.c[0] = v00.x; g.c[1] = v00.y; g.c[2] = v01.x; g.c[3] = v01.y;
    g.c[4] = v10.x; g.c[5] = v10.y; g.c[6] = v11.x; g.c[7] = v11.y;
    g.fl = ((xlo || xhi || (ix == 0 && ax == 0.0f)) ? 1u : 0u) | ((iy == 0 && g.ay == 0.0f) ? 2u : 0u) |
           ((iz == 0 && g.az == 0.0f) ? 4u : 0u);
}

// Value (and dvalue/dp) of a pending border-mode point; the same arithmetic
// as trilinear_clamped.
template <bool DERIV>
__device__ __forceinline__ Tri interp_pending(const Pend& g)
{
    const float e00 = g.c[1] - g.c[0], e01 = g.c[3] - g.c[2], e10 = g.c[5] - g.c[4], e11 = g.c[7] - g.c[6];
    const float c00 = fmaf(g.ax, e00, g.c[0]), c01 = fmaf(g.ax, e01, g.c[2]);
    const float c10 = fmaf(g.ax, e10, g.c[4]), c11 = fmaf(g.ax, e11, g.c[6]);
    const float f0 = c01 - c00, f1 = c11 - c10;
    const float c0 = fmaf(g.ay, f0, c00), c1 = fmaf(g.ay, f1, c10);
    Tri t;
    t.v = fmaf(g.az, c1 - c0, c0);
    if (DERIV) {
        const float gx0 = fmaf(g.ay, e01 - e00, e00), gx1 = fmaf(g.ay, e11 - e10, e10);
        t.dx = (g.fl & 1u) ? 0.0f : fmaf(g.az, gx1 - gx0, gx0);
        t.dy = (g.fl & 2u) ? 0.0f : fmaf(g.az, f1 - f0, f0);
        t.dz = (g.fl & 4u) ? 0.0f : (c1 - c0);
    } else {
        t.dx = t.dy = t.dz = 0.0f;
    }
    return t;
}

// Held to 128 VGPRs where 16 waves share a CU (1024-thread blocks, or two
// 512-thread blocks for windows up to 5); a 768-thread block is held to 168
// by its launch bound.  ADDR: see ld().
template <int WIN, int MODE, int PAD, int ADDR, int TX_, int TY_>
__global__ void __launch_bounds__(TX_ * TY_)
    __attribute__((amdgpu_waves_per_eu((TX_ * TY_ >= 1024 || WIN <= 5) ? 4 : 2, 8)))
lncc_kernel(LnccArgs a)
{
    using T = LnccTile<WIN, MODE, TX_, TY_>;
    constexpr int r = T::r, TX = T::TX, TY = T::TY, NT = T::NT;
    constexpr int R2 = T::R2, R1 = T::R1, X2 = T::X2, X1 = T::X1;
    constexpr int X1p = T::X1p, X2p = T::X2p;
    constexpr bool DER = (MODE != MODE_FWD);  // keep dMw/dp of the tile voxel
    constexpr float inv = 1.0f / float(WIN * WIN * WIN);
    __shared__ __attribute__((aligned(16))) float lds[T::LDS_FLOATS];
    float* sA = lds + T::OA;                   // [5][Y2][X2p]  z-window sums
    float* sB = lds + T::OB;                   // [5][Y2][X1p]  + x-window
    float* sC = sA;                            // [3][Y1][X1p]  a, c, e (aliases sA)
    float* sD = sB;                            // [3][Y1][TX]   x-window of a, c, e (aliases sB)
    float* sG = lds + T::OG;                   // [WIN][3][NT] dMw/dp of each thread's voxel
    double* sL = reinterpret_cast<double*>(lds + T::OL);  // [NT] loss accumulators (adjoint)

    const int D = a.D, H = a.H, W = a.W;
    const int HW = H * W;
    const size_t N = (size_t)D * HW;
    const int bid = xcd_remap(blockIdx.x, a.nblocks);
    const int tx = bid % a.ntx;
    const int rest = bid / a.ntx;
    const int ty = rest % a.nty;
    const int ch = rest / a.nty;
    const int gx0 = tx * TX, gy0 = ty * TY;
    const int z0 = ch * a.zchunk, z1 = min(D, z0 + a.zchunk);
    const int tid = threadIdx.x;

    // Window of the 32-bit addressing (ADDRWIN): zspan slices from zb, centred
    // on the slices the block streams (z0 - R2 - 1 .. z1 + R2); the launcher
    // guarantees zspan >= zchunk + 2 R2 + 4, so all of those lie inside.
    int zb = 0;
    if (ADDR == LNCC_ADDRWIN) {
        const int slack = a.zspan - (z1 - z0) - 2 * R2 - 4;
        zb = min(max(z0 - R2 - 2 - slack / 2, 0), max(D - a.zspan, 0));
    }
    const size_t wb = (size_t)zb * HW;  // element offset of the window
    const float* __restrict__ F = a.F;
    const float* __restrict__ M = a.M;
    const float* __restrict__ U = a.u;
    const float* __restrict__ Fb = F + wb;
    const float* __restrict__ Mb = M + wb;
    const float* __restrict__ U0 = U ? U + wb : nullptr;
    const float* __restrict__ U1 = U ? U + N + wb : nullptr;
    const float* __restrict__ U2 = U ? U + 2 * N + wb : nullptr;
    float* __restrict__ G0 = a.gu ? a.gu + wb : nullptr;
    float* __restrict__ G1 = a.gu ? a.gu + N + wb : nullptr;
    float* __restrict__ G2 = a.gu ? a.gu + 2 * N + wb : nullptr;

    // the thread's tile voxel (row iy, column ix) and halo-only stage-A points
    const int iy = tid / TX, ix = tid % TX;
    int hx[T::PH], hy[T::PH];
    // With at most one halo point per thread the NH halo points are spread
    // evenly over the waves (QW per wave, in the order top rows, bottom rows,
    // left and right side columns), so every wave samples about the same
    // number of points in stage A and reaches the following barrier together.
#pragma unroll
    for (int k = 0; k < T::PH; ++k) {
        int q;
        if (T::PH == 1) {
            const int wv = tid >> 6, ln = tid & 63;
            q = ln < T::QW ? wv * T::QW + ln : T::NH;
        } else {
            q = tid + k * NT;
        }
        hx[k] = -1; hy[k] = -1;
        if (q < T::NH) {
            if (q < R2 * X2) { hy[k] = q / X2; hx[k] = q - hy[k] * X2; }
            else if ((q -= R2 * X2) < R2 * X2) { hy[k] = R2 + TY + q / X2; hx[k] = q % X2; }
            else if ((q -= R2 * X2) < TY * R2) { hy[k] = R2 + q / R2; hx[k] = q % R2; }
            else { q -= TY * R2; hy[k] = R2 + q / R2; hx[k] = R2 + TX + q % R2; }
        }
    }

    // per-block shift: F and M at the tile centre
    const int sidx = (min((z0 + z1) / 2, D - 1) * H + min(gy0 + TY / 2, H - 1)) * W + min(gx0 + TX / 2, W - 1);
    const float sF = F[sidx], sM = M[sidx];
    const float gsc = a.grad_scale ? *a.grad_scale : 1.0f;
    const float gi = a.neg_inv_nroi * gsc;  // dL/dn_i on the ROI
    const float eps = a.eps;

    float rF[1 + T::PH][WIN], rM[1 + T::PH][WIN];  // shifted F, Mw: last w slices
    float zacc[MODE == MODE_BWD ? WIN : 1];        // pending outputs of the tile column
#pragma unroll
    for (int q = 0; q < (MODE == MODE_BWD ? WIN : 1); ++q) zacc[q] = 0.f;
    double lsum = 0.0;
    if (MODE == MODE_BWD) sL[tid] = 0.0;

    // stage-A points of this thread: k = 0 the tile voxel, k >= 1 halo points
    constexpr int P = 1 + T::PH;
    int pgx[P], pgy[P], pxy[P];
    bool pin[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int lx = k == 0 ? R2 + ix : hx[k - 1];
        const int ly = k == 0 ? R2 + iy : hy[k - 1];
        pgx[k] = gx0 - R2 + lx;
        pgy[k] = gy0 - R2 + ly;
        pin[k] = lx >= 0 && pgx[k] >= 0 && pgx[k] < W && pgy[k] >= 0 && pgy[k] < H;
        pxy[k] = pin[k] ? pgy[k] * W + pgx[k] : 0;
    }
    // Software pipeline over slices.  While slice zi is consumed, the loads
    // of slice zi+1 (F and, for border padding, the eight M corners) and u of
    // slice zi+2 are in flight, so HBM and L2 latency overlaps the LDS
    // stages.  Every load is in bounds (slice index clamped, off-array
    // points read voxel 0, corner indices clamped) and results are selected
    // when consumed.  Lanes without a halo point also sample (voxel 0, in
    // bounds) and only skip the LDS writes: branching around their loads
    // makes the compiler merge the pending registers of the skipped lanes
    // after the loads, which waits for the loads just issued (measured: the
    // w = 5 adjoint 10% faster on the 512^3 pair, w = 7 4%).
    float pu[P][3];
    Pend pend[P];
    auto load_u = [&](int zs, int k0, int k1) {
        const unsigned zoff = imul<ADDR>(min(max(zs, 0), D - 1) - zb, HW);
#pragma unroll
        for (int k = k0; k < k1; ++k) {
            if (U) {
                pu[k][0] = ld<ADDR>(U0, zoff + pxy[k]);
                pu[k][1] = ld<ADDR>(U1, zoff + pxy[k]);
                pu[k][2] = ld<ADDR>(U2, zoff + pxy[k]);
            } else {
                pu[k][0] = 0.f; pu[k][1] = 0.f; pu[k][2] = 0.f;
            }
        }
    };
    auto issue = [&](int zs, int k0, int k1) {  // uses pu = u of slice zs
        const unsigned zoff = imul<ADDR>(min(max(zs, 0), D - 1) - zb, HW);
#pragma unroll
        for (int k = k0; k < k1; ++k)
            issue_point<PAD, ADDR>(pend[k], M, Mb, Fb, D, H, W, HW, zb, a.zspan, pgx[k], pgy[k], zs,
                                   zoff + pxy[k], pu[k][0], pu[k][1], pu[k][2]);
    };
    // Schedule: the gathers of slice zi+1 are issued at the end of stage A of
    // slice zi, from u loaded two slices ahead.  Forward and ANTs kernels load
    // that u in stage C.  The adjoint kernel, whose registers are at the
    // limit, keeps every load out of stages B and C (the peak of register
    // pressure): its halo points load u of zi+1 at the start of stage D and
    // issue their gathers at the end of the slice (they are consumed after
    // the tile point in the next stage A), and the tile point's u of zi+2 is
    // loaded after those gathers.  (Measured on the adjoint: the u load in
    // stage C is 9% slower, at the start of stage D or E 8-10% slower, at the
    // start of stage A 3% slower.  The memory counter retires loads in
    // order, so where a load sits decides which waits it lengthens.)
    constexpr int KH = (MODE == MODE_BWD) ? 1 : P;  // points issued right after stage A
    load_u(z0 - R2, 0, P);
    issue(z0 - R2, 0, P);
    load_u(z0 - R2 + 1, 0, KH);

    const int nsteps = (z1 - z0) + 2 * R2;
    for (int base = 0; base < nsteps; base += WIN) {
#pragma unroll
        for (int j = 0; j < WIN; ++j) {
            const int s = base + j;
            if (s >= nsteps) break;
            const int zi = z0 - R2 + s;  // slice entering the rings
            const bool zin = (zi >= 0) && (zi < D);
            // ---- stage A: sample, push into the rings, z-window sums ----
            // Raised wave priority while the gathers of this slice are
            // consumed and those of the next are issued: the stage that ends
            // at the first barrier goes first, and the other block's LDS
            // stages fill the gaps (adjoint 4.5% faster than without).
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const bool act = k == 0 || hx[k - 1] >= 0;
                {
                    const bool ok = zin && pin[k];
                    float f = -sF, m = -sM;  // padded voxels are 0 before the shift
                    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
                    Tri t{0.f, 0.f, 0.f, 0.f};
                    if (PAD == PAD_BORDER) {
                        t = (DER && k == 0) ? interp_pending<DER>(pend[k]) : interp_pending<false>(pend[k]);
                    } else if (ok) {
                        t = (DER && k == 0)
                                ? trilinear<PAD_ZEROS, DER>(M, D, H, W, pgx[k], pgy[k], zi, pend[k].c[0], pend[k].c[1], pend[k].c[2])
                                : trilinear<PAD_ZEROS, false>(M, D, H, W, pgx[k], pgy[k], zi, pend[k].c[0], pend[k].c[1], pend[k].c[2]);
                    }
                    if (ok) {
                        f = pend[k].f - sF;
                        m = t.v - sM;
                        if (DER && k == 0) { d0 = t.dx; d1 = t.dy; d2 = t.dz; }
                    }
                    rF[k][j] = f;
                    rM[k][j] = m;
                    if (DER && k == 0) {
                        sG[(j * 3 + 0) * NT + tid] = d0;
                        sG[(j * 3 + 1) * NT + tid] = d1;
                        sG[(j * 3 + 2) * NT + tid] = d2;
                    }
                    if (s >= 2 * r && act) {
                        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
                        for (int q = 0; q < WIN; ++q) {
                            const float ff = rF[k][q], mm = rM[k][q];
                            s0 += ff;
                            s1 += mm;
                            s2 = fmaf(ff, ff, s2);
                            s3 = fmaf(mm, mm, s3);
                            s4 = fmaf(ff, mm, s4);
                        }
                        const int lx = k == 0 ? R2 + ix : hx[k - 1];
                        const int ly = k == 0 ? R2 + iy : hy[k - 1];
                        const int o = ly * X2p + lx;
                        sA[0 * T::NA + o] = s0;
                        sA[1 * T::NA + o] = s1;
                        sA[2 * T::NA + o] = s2;
                        sA[3 * T::NA + o] = s3;
                        sA[4 * T::NA + o] = s4;
                    }
                }
            }
            issue(zi + 1, 0, KH);
            __builtin_amdgcn_s_setprio(0);
            if (s < 2 * r) {  // rings not yet full (uniform over the block)
                load_u(zi + 2, 0, KH);
                if (KH < P) {
                    load_u(zi + 1, KH, P);
                    issue(zi + 1, KH, P);
                }
                continue;
            }
            __syncthreads();
            // ---- stage B: x-window, 2 outputs per thread ----
            for (int q = tid; q < T::RB; q += NT) {
                const int ly = q / (X1p / 2), lx0 = 2 * (q - ly * (X1p / 2));
#pragma unroll
                for (int c = 0; c < 5; ++c)
                    *reinterpret_cast<float2*>(sB + c * T::NB + ly * X1p + lx0) =
                        xwin2<WIN, T::NV>(sA + c * T::NA + ly * X2p + lx0);
            }
            __syncthreads();
            // ---- stage C: y-window, statistics, loss term, adjoint fields ----
            if (MODE != MODE_BWD) load_u(zi + 2, 0, KH);
            const int zc = zi - r;
            const bool zroi = zc >= a.roi[0] && zc < a.roi[1];
            const bool zown = zc >= z0 && zc < z1;
            if (MODE == MODE_BWD) {
                for (int q = tid; q < T::RC; q += NT) {
                    const int ly = q / (X1p / 2), lx0 = 2 * (q - ly * (X1p / 2));
                    float S[5][2];
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        float2 acc = *reinterpret_cast<const float2*>(sB + c * T::NB + ly * X1p + lx0);
#pragma unroll
                        for (int d = 1; d < WIN; ++d) {
                            const float2 t2 = *reinterpret_cast<const float2*>(sB + c * T::NB + (ly + d) * X1p + lx0);
                            acc.x += t2.x;
                            acc.y += t2.y;
                        }
                        S[c][0] = acc.x;
                        S[c][1] = acc.y;
                    }
                    const int gy = gy0 - R1 + ly;
                    const bool yroi = zroi && gy >= a.roi[2] && gy < a.roi[3];
                    const bool yown = zown && ly >= R1 && ly < R1 + TY;
                    float oa[2], oc[2], oe[2];
                    float lpart = 0.f;
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int lx = lx0 + e;
                        const int gx = gx0 - R1 + lx;
                        const bool inroi = yroi && lx < X1 && gx >= a.roi[4] && gx < a.roi[5];
                        const float mf = S[0][e] * inv, mm = S[1][e] * inv;
                        const float A = fmaf(-mf, mm, S[4][e] * inv);
                        const float B = fmaf(-mf, mf, S[2][e] * inv);
                        const float C = fmaf(-mm, mm, S[3][e] * inv);
                        const float rD = __builtin_amdgcn_rcpf(fmaf(B, C, eps));  // 1 ulp reciprocal
                        float ac = 0.f, cc = 0.f, ec = 0.f;
                        if (inroi) {
                            if (yown && lx >= R1 && lx < R1 + TX) lpart += A * A * rD;
                            ac = 2.0f * gi * A * rD;
                            cc = ac * A * B * rD;
                            ec = fmaf(cc, mm, -ac * mf);
                        }
                        oa[e] = ac; oc[e] = cc; oe[e] = ec;
                    }
                    if (lpart != 0.f) {
                        int t = tid;
                        asm volatile("" : "+v"(t));  // recompute the slot address here
                        sL[t] += (double)lpart;
                    }
                    const int o = ly * X1p + lx0;
                    *reinterpret_cast<float2*>(sC + 0 * T::NC + o) = make_float2(oa[0], oa[1]);
                    *reinterpret_cast<float2*>(sC + 1 * T::NC + o) = make_float2(oc[0], oc[1]);
                    *reinterpret_cast<float2*>(sC + 2 * T::NC + o) = make_float2(oe[0], oe[1]);
                }
            } else {
                // forward / ANTs: statistics at the thread's own tile voxel
                float S[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    float acc = 0.f;
#pragma unroll
                    for (int d = 0; d < WIN; ++d) acc += sB[c * T::NB + (iy + d) * X1p + ix];
                    S[c] = acc;
                }
                const int gx = gx0 + ix, gy = gy0 + iy;
                const bool inroi = zroi && gy >= a.roi[2] && gy < a.roi[3] && gx >= a.roi[4] && gx < a.roi[5];
                const float mf = S[0] * inv, mm = S[1] * inv;
                const float A = fmaf(-mf, mm, S[4] * inv);
                const float B = fmaf(-mf, mf, S[2] * inv);
                const float C = fmaf(-mm, mm, S[3] * inv);
                const float rD = __builtin_amdgcn_rcpf(fmaf(B, C, eps));  // 1 ulp reciprocal
                if (inroi && zown) lsum += (double)(A * A * rD);
                if (MODE == MODE_ANTS && zown && gx < W && gy < H) {
                    // gradient without the second window sum, at the voxel itself
                    const int sl = (j + WIN - r) % WIN;  // ring slot of slice zc
                    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
                    if (inroi) {
                        const float ac = 2.0f * gi * A * rD;
                        const float cc = ac * A * B * rD;
                        const float gm = ac * (rF[0][sl] - mf) - cc * (rM[0][sl] - mm);
                        g0 = gm * sG[(sl * 3 + 0) * NT + tid];
                        g1 = gm * sG[(sl * 3 + 1) * NT + tid];
                        g2 = gm * sG[(sl * 3 + 2) * NT + tid];
                    }
                    const unsigned idx = imul<ADDR>(zc - zb, HW) + imul<ADDR>(gy, W) + gx;
                    st<ADDR>(G0, idx, g0);
                    st<ADDR>(G1, idx, g1);
                    st<ADDR>(G2, idx, g2);
                }
            }
            if (MODE != MODE_BWD) continue;
            __syncthreads();
            load_u(zi + 1, KH, P);
            // ---- stage D: x-window of a, c, e ----
            for (int q = tid; q < T::RD; q += NT) {
                const int ly = q / (TX / 2), lx0 = 2 * (q - ly * (TX / 2));
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    *reinterpret_cast<float2*>(sD + c * T::ND + ly * TX + lx0) =
                        xwin2<WIN, T::NV>(sC + c * T::NC + ly * X1p + lx0);
            }
            __syncthreads();
            // ---- stages E/F: y-window, z-window by scatter, gradient ----
            // The xy-windowed a, c, e of slice zc enter the pending outputs
            // zo = zc - r .. zc + r of the thread's column, each as
            // F(zo) a - Mw(zo) c + e with that output's own (shifted) F and Mw
            // from the ring, so the z-window needs one accumulator per pending
            // output slice instead of a ring per field.
            {
                const int zo = zc - r;
                const int so = (j + 1) % WIN;  // ring slot of slice zo (the oldest)
                float ya = 0.f, yc = 0.f, ye = 0.f;
#pragma unroll
                for (int d = 0; d < WIN; ++d) {
                    ya += sD[0 * T::ND + (iy + d) * TX + ix];
                    yc += sD[1 * T::ND + (iy + d) * TX + ix];
                    ye += sD[2 * T::ND + (iy + d) * TX + ix];
                }
#pragma unroll
                for (int q = 0; q < WIN; ++q) zacc[q] = fmaf(rF[0][q], ya, fmaf(-rM[0][q], yc, zacc[q] + ye));
                const int gx = gx0 + ix, gy = gy0 + iy;
                if (s >= 4 * r && zo >= z0 && zo < z1 && gx < W && gy < H) {
                    const float gm = zacc[so] * inv;
                    const unsigned idx = imul<ADDR>(zo - zb, HW) + imul<ADDR>(gy, W) + gx;
                    st<ADDR>(G0, idx, gm * sG[(so * 3 + 0) * NT + tid]);
                    st<ADDR>(G1, idx, gm * sG[(so * 3 + 1) * NT + tid]);
                    st<ADDR>(G2, idx, gm * sG[(so * 3 + 2) * NT + tid]);
                }
                zacc[so] = 0.f;  // the slot of the next new pending output
            }
            issue(zi + 1, KH, P);
            load_u(zi + 2, 0, KH);
        }
    }
    // ---- block loss partial (fixed-order tree) ----
    __syncthreads();
    if (MODE == MODE_BWD) lsum = sL[tid];
    double tot = block_sum<NT>(lsum, reinterpret_cast<double*>(lds));
    if (tid == 0) a.partial[blockIdx.x] = tot;
}

// loss = 1 - sum(partials) / N_roi, summed in a fixed order
__global__ void __launch_bounds__(256) lncc_finalize(const double* __restrict__ partial, int n, double inv_nroi,
                                                     float* loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) *loss = (float)(1.0 - s * inv_nroi);
}

// Tile of a (window, mode): 32 x 16 columns, 512 threads.  (Measured: a
// 32 x 32 tile with 1024 threads, which samples 1.56 instead of 1.88 points
// per output at w = 5, runs one block per CU and spills registers at the
// 128-VGPR limit; the adjoint took 3.72 ms against 2.81 ms at 512^3.)
// Column tile of a launch: 32 x 16 (512 threads), except the w = 7 adjoint,
// 32 x 24 (768 threads).  At w = 7 the 16-row tile samples 2.41 points per
// output (its 4r halo) and its 167 VGPRs and 96 KB of LDS leave one block of
// 8 waves per CU; 24 rows sample 2.06 points per output, and one block of
// 12 waves fits (168 VGPRs, 134 KB): 512^3 adjoint 5.10 -> 4.74 ms, 1040^3
// 45.6 -> 38.2 ms.  (32 x 32 does not fit the LDS; at w = 5 the two-block
// 32 x 16 layout stays faster than any one-block tile.)
static void lncc_tile(int win, int mode, int& tx, int& ty)
{
    tx = 32;
    ty = (win == 7 && mode == MODE_BWD) ? 24 : 16;
}

LnccLaunch lncc_plan(int D, int H, int W, int win, int mode)
{
    LnccLaunch L;
    lncc_tile(win, mode, L.tx, L.ty);
    L.nt = L.tx * L.ty;
    const int r = (win - 1) / 2;
    const int R2 = (mode == MODE_BWD) ? 2 * r : r;
    L.ntx = (W + L.tx - 1) / L.tx;
    L.nty = (H + L.ty - 1) / L.ty;
    const long long tiles = (long long)L.ntx * L.nty;
    // z-chunks: blocks are dispatched as CUs free up, so the run ends after
    // ceil(nblocks / slots) block times of (zchunk + 2 R2) slices each (slots
    // = resident blocks on 256 CUs).  Take the chunk count (z-chunks of at
    // least 16 slices) that minimises that estimate; ties go to fewer chunks.
    const long long slots = 256LL * (L.nt >= 1024 ? 1 : ((win <= 5) ? 2 : 1));
    const int maxchunks = max(1, D / 16);
    long long best = -1;
    int bc = 1;
    for (int c = 1; c <= maxchunks && c <= 64; ++c) {
        const int zc = (D + c - 1) / c;
        const int nc = (D + zc - 1) / zc;
        const long long rounds = (tiles * nc + slots - 1) / slots;
        const long long cost = rounds * (zc + 2 * R2);
        if (best < 0 || cost < best) { best = cost; bc = c; }
    }
    L.zchunk = (D + bc - 1) / bc;
    L.nchunks = (D + L.zchunk - 1) / L.zchunk;
    L.nblocks = (int)(tiles * L.nchunks);
    // addressing: 32-bit byte offsets where the volume (or a window of
    // slices around each block) stays below 4 GB and index factors fit 24 bits
    const long long N = (long long)D * H * W;
    const long long HW = (long long)H * W;
    const bool fit24 = D < (1 << 24) && HW < (1 << 24);
    const long long span = 4294967295LL / (4 * HW);  // whole slices within 4 GB of a base
    L.zspan = (int)min(span, (long long)D);
    if (W >= 2 && fit24 && N * 4 <= 4294967295LL) L.addr = LNCC_ADDR32;
    else if (W >= 2 && fit24 && span >= L.zchunk + 2 * R2 + 4) L.addr = LNCC_ADDRWIN;
    else L.addr = LNCC_ADDR64;  // also width-1 volumes (no x pairs)
    return L;
}

int lncc_max_blocks(int D, int H, int W, int win)
{
    int n = 0;
    for (int mode = 0; mode < 3; ++mode) n = max(n, lncc_plan(D, H, W, win, mode).nblocks);
    return n;
}

template <int WIN, int MODE, int TX, int TY>
static hipError_t launch_t(int pad, int addr, const LnccArgs& a, hipStream_t st)
{
    dim3 grid(a.nblocks), block(TX * TY);
    if (pad == PAD_BORDER) {
        if (addr == LNCC_ADDR32)
            hipLaunchKernelGGL((lncc_kernel<WIN, MODE, PAD_BORDER, LNCC_ADDR32, TX, TY>), grid, block, 0, st, a);
        else if (addr == LNCC_ADDRWIN)
            hipLaunchKernelGGL((lncc_kernel<WIN, MODE, PAD_BORDER, LNCC_ADDRWIN, TX, TY>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((lncc_kernel<WIN, MODE, PAD_BORDER, LNCC_ADDR64, TX, TY>), grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL((lncc_kernel<WIN, MODE, PAD_ZEROS, LNCC_ADDR64, TX, TY>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

template <int WIN, int MODE>
static hipError_t launch_w(int pad, const LnccLaunch& L, const LnccArgs& a, hipStream_t st)
{
    if constexpr (WIN == 7 && MODE == MODE_BWD) {
        if (L.tx != 32 || L.ty != 24) return hipErrorInvalidValue;
        return launch_t<WIN, MODE, 32, 24>(pad, L.addr, a, st);
    } else {
        if (L.tx != 32 || L.ty != 16) return hipErrorInvalidValue;
        return launch_t<WIN, MODE, 32, 16>(pad, L.addr, a, st);
    }
}

template <int MODE>
static hipError_t launch_mode(int win, int pad, const LnccLaunch& L, const LnccArgs& a, hipStream_t st)
{
    switch (win) {
        case 3: return launch_w<3, MODE>(pad, L, a, st);
        case 5: return launch_w<5, MODE>(pad, L, a, st);
        case 7: return launch_w<7, MODE>(pad, L, a, st);
        case 9: return launch_w<9, MODE>(pad, L, a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t lncc_launch(int mode, int win, int pad, const LnccLaunch& L, const LnccArgs& a, float* loss, double nroi,
                       hipStream_t st)
{
    hipError_t e;
    if (mode == MODE_FWD) e = launch_mode<MODE_FWD>(win, pad, L, a, st);
    else if (mode == MODE_BWD) e = launch_mode<MODE_BWD>(win, pad, L, a, st);
    else e = launch_mode<MODE_ANTS>(win, pad, L, a, st);
    if (e != hipSuccess) return e;
    if (loss) {
        hipLaunchKernelGGL(lncc_finalize, dim3(1), dim3(256), 0, st, a.partial, a.nblocks, 1.0 / nroi, loss);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace ffdp
