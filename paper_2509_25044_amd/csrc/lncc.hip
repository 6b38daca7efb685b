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
//  * a block owns a TX x TY column tile and a z-chunk, and streams z slices;
//  * stage A samples F and Mw on the tile plus a halo of 2r (r for the
//    forward), keeping the last w slices per column in registers, and writes
//    the five z-window sums to LDS;
//  * stages B/C finish the separable box in x then y, form A, B, C and the
//    loss term, then a, c, e; stages D/E box a, c, e in x, y and (via a
//    register ring) z; stage F re-samples Mw with its derivative at the output
//    voxel and writes grad_u.  Interpolation weights are recomputed, never stored.
//  * all statistics use values shifted by a per-block constant (F and M at
//    the tile centre).  With the padded voxels shifted too, A, B, C and the
//    adjoint are unchanged in exact arithmetic, and the fp32 cancellation in
//    B = mu_FF - mu_F^2 shrinks.
//  * window sums are direct w-term sums (no running add/subtract drift).
#include "device.hpp"
#include "internal.hpp"

namespace ffdp {

enum { MODE_FWD = 0, MODE_BWD = 1, MODE_ANTS = 2 };

template <int WIN, int MODE>
struct LnccTile {
    static constexpr int r = (WIN - 1) / 2;
    static constexpr int TX = LNCC_TX, TY = LNCC_TY, NT = LNCC_NT;
    static constexpr int R2 = (MODE == MODE_BWD) ? 2 * r : r;  // stage-A halo
    static constexpr int R1 = (MODE == MODE_BWD) ? r : 0;      // stage-C halo
    static constexpr int X2 = TX + 2 * R2, Y2 = TY + 2 * R2;
    static constexpr int X1 = TX + 2 * R1, Y1 = TY + 2 * R1;
    static constexpr int NA = X2 * Y2;  // stage A points
    static constexpr int NB = Y2 * X1;  // x-box outputs
    static constexpr int NC = X1 * Y1;  // statistic points
    static constexpr int ND = Y1 * TX;  // x-box of the adjoint fields
    static constexpr int NE = TX * TY;  // output points
    static constexpr int PA = (NA + NT - 1) / NT;
    static constexpr int PE = (NE + NT - 1) / NT;
    static constexpr int LDS_FLOATS = 5 * NA + 5 * NB;
};

template <int WIN, int MODE, int PAD>
__global__ void __launch_bounds__(LNCC_NT) lncc_kernel(LnccArgs a)
{
    using T = LnccTile<WIN, MODE>;
    constexpr int r = T::r, TX = T::TX, TY = T::TY, NT = T::NT;
    constexpr int R2 = T::R2, R1 = T::R1, X2 = T::X2, X1 = T::X1;
    constexpr float inv = 1.0f / float(WIN * WIN * WIN);
    __shared__ float lds[T::LDS_FLOATS];
    float* sA = lds;               // [5][NA]  z-window sums on the stage-A points
    float* sB = lds + 5 * T::NA;   // [5][NB]  x-box
    float* sC = lds;               // [3][NC]  a, c, e (aliases sA)
    float* sD = lds + 5 * T::NA;   // [3][ND]  x-box of a, c, e (aliases sB)

    const int D = a.D, H = a.H, W = a.W;
    const int HW = H * W;
    const int bid = xcd_remap(blockIdx.x, a.nblocks);
    const int tx = bid % a.ntx;
    const int rest = bid / a.ntx;
    const int ty = rest % a.nty;
    const int ch = rest / a.nty;
    const int gx0 = tx * TX, gy0 = ty * TY;
    const int z0 = ch * a.zchunk, z1 = min(D, z0 + a.zchunk);
    const int tid = threadIdx.x;

    const float* __restrict__ F = a.F;
    const float* __restrict__ M = a.M;
    const float* __restrict__ u0 = a.u;
    const float* __restrict__ u1 = a.u ? a.u + (size_t)D * HW : nullptr;
    const float* __restrict__ u2 = a.u ? a.u + 2 * (size_t)D * HW : nullptr;

    // per-block shift: F and M at the tile centre
    const int sidx = (min((z0 + z1) / 2, D - 1) * H + min(gy0 + TY / 2, H - 1)) * W + min(gx0 + TX / 2, W - 1);
    const float sF = F[sidx], sM = M[sidx];
    const float gsc = a.grad_scale ? *a.grad_scale : 1.0f;
    const float gi = a.neg_inv_nroi * gsc;  // dL/dn_i on the ROI
    const float eps = a.eps;

    float rF[T::PA][WIN], rM[T::PA][WIN];  // raw shifted samples, last w slices
    float rE[3][T::PE][WIN];               // xy-boxed a, c, e, last w slices
    double lsum = 0.0;

    const int nsteps = (z1 - z0) + 2 * R2;
    for (int base = 0; base < nsteps; base += WIN) {
#pragma unroll
        for (int j = 0; j < WIN; ++j) {
            const int s = base + j;
            if (s >= nsteps) break;
            const int zi = z0 - R2 + s;  // slice entering the ring
            const bool zin = (zi >= 0) && (zi < D);
            // ---- stage A: sample, push into the ring, z-window sums ----
#pragma unroll
            for (int k = 0; k < T::PA; ++k) {
                const int p = tid + k * NT;
                if (p < T::NA) {
                    const int ly = p / X2, lx = p - ly * X2;
                    const int gx = gx0 - R2 + lx, gy = gy0 - R2 + ly;
                    float f = -sF, m = -sM;  // padded voxels are 0 before the shift
                    if (zin && gx >= 0 && gx < W && gy >= 0 && gy < H) {
                        const int idx = zi * HW + gy * W + gx;
                        float ux = 0.f, uy = 0.f, uz = 0.f;
                        if (u0) { ux = u0[idx]; uy = u1[idx]; uz = u2[idx]; }
                        f = F[idx] - sF;
                        m = trilinear<PAD, false>(M, D, H, W, gx, gy, zi, ux, uy, uz).v - sM;
                    }
                    rF[k][j] = f;
                    rM[k][j] = m;
                    if (s >= 2 * r) {
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
                        sA[0 * T::NA + p] = s0;
                        sA[1 * T::NA + p] = s1;
                        sA[2 * T::NA + p] = s2;
                        sA[3 * T::NA + p] = s3;
                        sA[4 * T::NA + p] = s4;
                    }
                }
            }
            if (s < 2 * r) continue;  // ring not yet full (uniform over the block)
            __syncthreads();
            // ---- stage B: x-box ----
            for (int p = tid; p < T::NB; p += NT) {
                const int ly = p / X1, lx = p - ly * X1;
                const int b0 = ly * X2 + lx;
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    float acc = 0.f;
#pragma unroll
                    for (int d = 0; d < WIN; ++d) acc += sA[c * T::NA + b0 + d];
                    sB[c * T::NB + p] = acc;
                }
            }
            __syncthreads();
            // ---- stage C: y-box, statistics, loss term, adjoint fields ----
            const int zc = zi - r;
            for (int p = tid; p < T::NC; p += NT) {
                const int ly = p / X1, lx = p - ly * X1;
                float S[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    float acc = 0.f;
#pragma unroll
                    for (int d = 0; d < WIN; ++d) acc += sB[c * T::NB + (ly + d) * X1 + lx];
                    S[c] = acc;
                }
                const int gx = gx0 - R1 + lx, gy = gy0 - R1 + ly;
                const bool inroi = zc >= a.roi[0] && zc < a.roi[1] && gy >= a.roi[2] && gy < a.roi[3] &&
                                   gx >= a.roi[4] && gx < a.roi[5];
                const bool owned = lx >= R1 && lx < R1 + TX && ly >= R1 && ly < R1 + TY && zc >= z0 && zc < z1;
                const float mf = S[0] * inv, mm = S[1] * inv;
                const float A = fmaf(-mf, mm, S[4] * inv);
                const float B = fmaf(-mf, mf, S[2] * inv);
                const float C = fmaf(-mm, mm, S[3] * inv);
                const float Dn = fmaf(B, C, eps);
                if (inroi && owned) lsum += (double)(A * A / Dn);
                if (MODE == MODE_BWD) {
                    float ac = 0.f, cc = 0.f, ec = 0.f;
                    if (inroi) {
                        ac = 2.0f * gi * A / Dn;
                        cc = ac * A * B / Dn;
                        ec = fmaf(cc, mm, -ac * mf);
                    }
                    sC[0 * T::NC + p] = ac;
                    sC[1 * T::NC + p] = cc;
                    sC[2 * T::NC + p] = ec;
                }
                if (MODE == MODE_ANTS && owned && gx < W && gy < H) {
                    // gradient without the second window sum, at the voxel itself
                    const int idx = zc * HW + gy * W + gx;
                    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
                    if (inroi) {
                        float ux = 0.f, uy = 0.f, uz = 0.f;
                        if (u0) { ux = u0[idx]; uy = u1[idx]; uz = u2[idx]; }
                        const Tri t = trilinear<PAD, true>(M, D, H, W, gx, gy, zc, ux, uy, uz);
                        const float ac = 2.0f * gi * A / Dn;
                        const float cc = ac * A * B / Dn;
                        const float gm = ac * ((F[idx] - sF) - mf) - cc * ((t.v - sM) - mm);
                        g0 = gm * t.dx; g1 = gm * t.dy; g2 = gm * t.dz;
                    }
                    a.gu[idx] = g0;
                    a.gu[(size_t)D * HW + idx] = g1;
                    a.gu[2 * (size_t)D * HW + idx] = g2;
                }
            }
            if (MODE != MODE_BWD) continue;
            __syncthreads();
            // ---- stage D: x-box of a, c, e ----
            for (int p = tid; p < T::ND; p += NT) {
                const int ly = p / TX, lx = p - ly * TX;
                const int b0 = ly * X1 + lx;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float acc = 0.f;
#pragma unroll
                    for (int d = 0; d < WIN; ++d) acc += sC[c * T::NC + b0 + d];
                    sD[c * T::ND + p] = acc;
                }
            }
            __syncthreads();
            // ---- stages E/F: y-box into the register ring, z-box, gradient ----
            const int zo = zc - r;
#pragma unroll
            for (int k = 0; k < T::PE; ++k) {
                const int p = tid + k * NT;
                if (p < T::NE) {
                    const int ly = p / TX, lx = p - ly * TX;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float acc = 0.f;
#pragma unroll
                        for (int d = 0; d < WIN; ++d) acc += sD[c * T::ND + (ly + d) * TX + lx];
                        rE[c][k][j] = acc;
                    }
                    const int gx = gx0 + lx, gy = gy0 + ly;
                    if (s >= 4 * r && zo >= z0 && zo < z1 && gx < W && gy < H) {
                        float ba = 0.f, bc = 0.f, be = 0.f;
#pragma unroll
                        for (int q = 0; q < WIN; ++q) {
                            ba += rE[0][k][q];
                            bc += rE[1][k][q];
                            be += rE[2][k][q];
                        }
                        const int idx = zo * HW + gy * W + gx;
                        float ux = 0.f, uy = 0.f, uz = 0.f;
                        if (u0) { ux = u0[idx]; uy = u1[idx]; uz = u2[idx]; }
                        const Tri t = trilinear<PAD, true>(M, D, H, W, gx, gy, zo, ux, uy, uz);
                        const float gm = ((F[idx] - sF) * ba - (t.v - sM) * bc + be) * inv;
                        a.gu[idx] = gm * t.dx;
                        a.gu[(size_t)D * HW + idx] = gm * t.dy;
                        a.gu[2 * (size_t)D * HW + idx] = gm * t.dz;
                    }
                }
            }
        }
    }
    // ---- block loss partial (fixed-order tree) ----
    __syncthreads();
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

LnccLaunch lncc_plan(int D, int H, int W)
{
    // Enough blocks to fill 256 CUs (about 1024), but z-chunks of at least 64
    // slices where the volume allows, so the 2r..4r recomputed halo slices stay
    // a small fraction of the streamed slices.
    LnccLaunch L;
    L.ntx = (W + LNCC_TX - 1) / LNCC_TX;
    L.nty = (H + LNCC_TY - 1) / LNCC_TY;
    const int tiles = L.ntx * L.nty;
    int chunks = (1024 + tiles - 1) / tiles;
    const int maxchunks = (D + 63) / 64;
    if (chunks > maxchunks) chunks = maxchunks;
    if (chunks < 1) chunks = 1;
    L.zchunk = (D + chunks - 1) / chunks;
    L.nchunks = (D + L.zchunk - 1) / L.zchunk;
    L.nblocks = tiles * L.nchunks;
    return L;
}

template <int WIN, int MODE>
static hipError_t launch_w(int pad, const LnccArgs& a, hipStream_t st)
{
    dim3 grid(a.nblocks), block(LNCC_NT);
    if (pad == PAD_BORDER)
        hipLaunchKernelGGL((lncc_kernel<WIN, MODE, PAD_BORDER>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((lncc_kernel<WIN, MODE, PAD_ZEROS>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(int win, int pad, const LnccArgs& a, hipStream_t st)
{
    switch (win) {
        case 3: return launch_w<3, MODE>(pad, a, st);
        case 5: return launch_w<5, MODE>(pad, a, st);
        case 7: return launch_w<7, MODE>(pad, a, st);
        case 9: return launch_w<9, MODE>(pad, a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t lncc_launch(int mode, int win, int pad, const LnccArgs& a, float* loss, double nroi, hipStream_t st)
{
    hipError_t e;
    if (mode == MODE_FWD) e = launch_mode<MODE_FWD>(win, pad, a, st);
    else if (mode == MODE_BWD) e = launch_mode<MODE_BWD>(win, pad, a, st);
    else e = launch_mode<MODE_ANTS>(win, pad, a, st);
    if (e != hipSuccess) return e;
    if (loss) {
        hipLaunchKernelGGL(lncc_finalize, dim3(1), dim3(256), 0, st, a.partial, a.nblocks, 1.0 / nroi, loss);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace ffdp
