// Fused warp + Parzen-window mutual information for gfx950.
//
// What is computed (eq. mi; App. "Implicit MI implementation"):
//   p[m][n] = (1/N_roi) sum_{k in ROI} kappa_m(F_k) kappa_n(Mw_k),  Mw = M(x+u)
//   MI = sum p log(p / (p_F p_M)),  loss = -MI
//   dloss/dMw_k = -(1/N_roi) sum_{m,n} kappa_m(F_k) omega_n(Mw_k) T[m][n],
//   T[m][n] = log p[m][n] - log p_M[n]
// kappa_m(v) = beta3(s - m), s = clamp(v,0,1) B - 1/2, the cubic B-spline
// over one bin width, support beyond the edge bins folded onto them;
// omega = d kappa / dv.  The full derivative of MI with respect to p also has
// the terms -log p_F[m] - 1, which drop out because sum_n omega_n = 0 (the
// kernel is a partition of unity).
//
// Forward: no Parzen block is materialised (the paper's point).  Each voxel
// touches a 4 x 4 patch of the joint histogram.  A thread walks one (x, y)
// column along z; consecutive voxels of a smooth volume usually share the
// same 4 x 4 patch, so the thread accumulates the patch in registers and
// flushes it to an LDS histogram only when the patch moves.  LDS and global
// histograms hold unsigned 64-bit fixed point (2^-32 units): integer atomics
// commute, so the histogram is bitwise reproducible.  Neighbouring voxels
// have similar intensities and so hit the same bins; to keep the lanes of a
// wave from serialising on one address, a block keeps several LDS copies of
// its histogram and neighbouring lanes add into different copies.  A
// one-block kernel then forms p, the marginals, MI and the log table T.
// Backward: T in LDS, 4 x 4 weighted lookups per voxel, then the sampler's
// derivative; grad_u written over the whole array (zero outside the ROI).
//
// Approximate forward (App. "Implicit MI implementation", the approximate
// histogram estimator): each voxel adds one count to its hard bin pair
// (min(floor(v B), B-1) of the exact product) -- runs of equal bin pairs along a column
// are merged in a register before the LDS atomic -- and the one-block
// finalize convolves the count histogram with the kernel at bin-centre
// offsets (taps 1/6, 2/3, 1/6, folded at the edges) before forming p.  Its
// backward is the exact one above, fed with the approximate p.
#include "device.hpp"
#include "internal.hpp"

namespace ffdp {

// Border padding of a volume one column wide: the x corners are loaded one
// by one (PAD_BORDER loads them as one 8-byte pair, which needs W >= 2).
constexpr int MI_PAD_BORDER1 = 2;

// Hard bin min(floor(v B), B-1) of a value v in [0, 1], taken on the exact
// product v B rather than its fp32 rounding: p = fl(v B) and its residual
// fma(v, B, -p) is exact, so floor(v B) = floor(p) except where p is an
// integer reached by rounding up (residual < 0).  The decision is then the
// same as floor in any wider precision for the same fp32 v.
__device__ __forceinline__ int exact_bin(float vc, int B)
{
    const float fB = (float)B;
    const float p = vc * fB;
    const float e = fmaf(vc, fB, -p);
    float f = floorf(p);
    if (f == p && e < 0.0f) f -= 1.0f;
    return min((int)f, B - 1);
}

// Four cubic B-spline weights of v on bins j0..j0+3 (before folding) and, with
// DERIV, their derivatives with respect to v.  Hard mode: one unit weight.
template <bool HARD, bool DERIV>
__device__ __forceinline__ void parzen4(float v, int B, int& j0, float w[4], float dw[4])
{
    const float vc = fminf(fmaxf(v, 0.0f), 1.0f);  // NaN -> 0; flagged separately
    if (HARD) {
        j0 = exact_bin(vc, B);
        w[0] = 1.0f; w[1] = w[2] = w[3] = 0.0f;
        if (DERIV) dw[0] = dw[1] = dw[2] = dw[3] = 0.0f;
        return;
    }
    const float s = vc * (float)B - 0.5f;
    const float f = floorf(s);
    const float t = s - f, q = 1.0f - t;
    j0 = (int)f - 1;
    const float t2 = t * t, q2 = q * q;
    w[0] = q2 * q * (1.0f / 6.0f);
    w[1] = fmaf(0.5f * t, t2, 2.0f / 3.0f - t2);
    w[2] = fmaf(0.5f * q, q2, 2.0f / 3.0f - q2);
    w[3] = t2 * t * (1.0f / 6.0f);
    if (DERIV) {
        const float ds = (v >= 0.0f && v <= 1.0f) ? (float)B : 0.0f;
        dw[0] = -0.5f * q2 * ds;
        dw[1] = fmaf(1.5f, t2, -2.0f * t) * ds;
        dw[2] = fmaf(-1.5f, q2, 2.0f * q) * ds;
        dw[3] = 0.5f * t2 * ds;
    }
}

__device__ __forceinline__ int fold(int j, int B) { return min(max(j, 0), B - 1); }

// Offset from voxel (x, y, z) to its sample point: u, or with the composite
// sampler Am X + t + S u.
template <bool AFF>
__device__ __forceinline__ void sample_disp(const MiArgs& a, int x, int y, int z, int idx, size_t N, float& dx,
                                            float& dy, float& dz)
{
    float ux = 0.f, uy = 0.f, uz = 0.f;
    if (a.u) { ux = a.u[idx]; uy = a.u[N + idx]; uz = a.u[2 * N + idx]; }
    if (AFF) affine_disp(a.aff, x, y, z, ux, uy, uz, dx, dy, dz);
    else { dx = ux; dy = uy; dz = uz; }
}

// round(x 2^32) for 0 <= x < 2^24 in fp32 and integer steps: the integer part
// hi, then the fraction f = x - hi (exact) scaled by 2^32 (exact) plus 1/2
// and truncated.  Where x >= 2^-9, f is a multiple of 2^-32, so f 2^32 is an
// integer and the rounding of the + 1/2 can move it by at most one unit
// (2^-32 of a voxel); below, f 2^32 + 1/2 is exact and the result is the
// rounded value.  The same input always gives the same integer.
__device__ __forceinline__ unsigned long long to_fix(float x)
{
    const unsigned hi = (unsigned)x;
    // x - floor(x) in one instruction (exact for x >= 0, the same value as
    // x - (float)hi)
    const unsigned lo = (unsigned)fmaf(__builtin_amdgcn_fractf(x), 4294967296.0f, 0.5f);
    return ((unsigned long long)hi << 32) | lo;
}

// Loads of one voxel's sample, issued one z-step ahead of their use (the
// thread walks its column along z): F, the eight corner values of M's cell
// (indices clamped into the array, so every load is in bounds), the cell
// fractions, and flags.  Border padding: a flag per axis for a sample exactly
// on index 0 (zero derivative there, as trilinear<PAD_BORDER>; the clamped
// corners make value and derivative right elsewhere).  Zero padding: one
// validity bit per corner, applied when the values are consumed.
typedef float mi_f2a __attribute__((ext_vector_type(2), aligned(4)));  // 4-byte aligned pair: one 8-byte load

struct MiPend {
    float c[8];
    float ax, ay, az;
    unsigned fl;
    float f;
};

template <int PAD>
__device__ __forceinline__ void mi_issue(const MiArgs& a, int x, int y, int z, float dx, float dy, float dz, int idx,
                                         MiPend& g)
{
    const int D = a.D, H = a.H, W = a.W;
    g.f = __builtin_nontemporal_load(a.F + idx);  // read once per kernel
    const float fx = fminf(fmaxf(floorf(dx), -268435456.0f), 268435456.0f);
    const float fy = fminf(fmaxf(floorf(dy), -268435456.0f), 268435456.0f);
    const float fz = fminf(fmaxf(floorf(dz), -268435456.0f), 268435456.0f);
    g.ax = dx - fx; g.ay = dy - fy; g.az = dz - fz;
    const int ix = x + (int)fx, iy = y + (int)fy, iz = z + (int)fz;
    const int y0 = min(max(iy, 0), H - 1), y1 = min(max(iy + 1, 0), H - 1);
    const int z0 = min(max(iz, 0), D - 1), z1 = min(max(iz + 1, 0), D - 1);
    const int r00 = (z0 * H + y0) * W, r01 = (z0 * H + y1) * W, r10 = (z1 * H + y0) * W, r11 = (z1 * H + y1) * W;
    if (PAD == PAD_BORDER) {  // W >= 2 (single columns run MI_PAD_BORDER1)
        // x corners: one 8-byte load of columns xp, xp + 1; a point clamped
        // at the low border takes the first of the pair (weight 0), at the
        // high border the second (weight 1, equal to it up to one rounding),
        // with a zero x derivative either way (flag bit 0)
        const bool xlo = ix < 0, xhi = ix >= W - 1;
        const int xp = min(max(ix, 0), W - 2);
        const float ax = g.ax;
        g.ax = xlo ? 0.0f : (xhi ? 1.0f : ax);
        const mi_f2a v00 = *reinterpret_cast<const mi_f2a*>(a.M + r00 + xp);
        const mi_f2a v01 = *reinterpret_cast<const mi_f2a*>(a.M + r01 + xp);
        const mi_f2a v10 = *reinterpret_cast<const mi_f2a*>(a.M + r10 + xp);
        const mi_f2a v11 = *reinterpret_cast<const mi_f2a*>(a.M + r11 + xp);
        g.c[0] = v00.x; g.c[1] = v00.y; g.c[2] = v01.x; g.c[3] = v01.y;
        g.c[4] = v10.x; g.c[5] = v10.y; g.c[6] = v11.x; g.c[7] = v11.y;
        g.fl = ((xlo || xhi || (ix == 0 && ax == 0.0f)) ? 1u : 0u) | ((iy == 0 && g.ay == 0.0f) ? 2u : 0u) |
               ((iz == 0 && g.az == 0.0f) ? 4u : 0u);
        return;
    }
    const int x0 = min(max(ix, 0), W - 1), x1 = min(max(ix + 1, 0), W - 1);
    g.c[0] = a.M[r00 + x0]; g.c[1] = a.M[r00 + x1]; g.c[2] = a.M[r01 + x0]; g.c[3] = a.M[r01 + x1];
    g.c[4] = a.M[r10 + x0]; g.c[5] = a.M[r10 + x1]; g.c[6] = a.M[r11 + x0]; g.c[7] = a.M[r11 + x1];
    if (PAD == MI_PAD_BORDER1) {
        g.fl = ((ix == 0 && g.ax == 0.0f) ? 1u : 0u) | ((iy == 0 && g.ay == 0.0f) ? 2u : 0u) |
               ((iz == 0 && g.az == 0.0f) ? 4u : 0u);
    } else {
        unsigned m = 0u;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int cx = ix + (b & 1), cy = iy + ((b >> 1) & 1), cz = iz + (b >> 2);
            if ((unsigned)cx < (unsigned)W && (unsigned)cy < (unsigned)H && (unsigned)cz < (unsigned)D) m |= 1u << b;
        }
        g.fl = m;
    }
}

// Value and (with DERIV) dvalue/dp of a pending sample; the arithmetic of
// trilinear<PAD, DERIV>.
template <int PAD, bool DERIV>
__device__ __forceinline__ Tri mi_interp(const MiPend& g)
{
    float c[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) c[b] = (PAD == PAD_ZEROS && !((g.fl >> b) & 1u)) ? 0.0f : g.c[b];
    const float e00 = c[1] - c[0], e01 = c[3] - c[2], e10 = c[5] - c[4], e11 = c[7] - c[6];
    const float c00 = fmaf(g.ax, e00, c[0]), c01 = fmaf(g.ax, e01, c[2]);
    const float c10 = fmaf(g.ax, e10, c[4]), c11 = fmaf(g.ax, e11, c[6]);
    const float f0 = c01 - c00, f1 = c11 - c10;
    const float c0 = fmaf(g.ay, f0, c00), c1 = fmaf(g.ay, f1, c10);
    Tri t;
    t.v = fmaf(g.az, c1 - c0, c0);
    if (DERIV) {
        const bool bx = PAD != PAD_ZEROS && (g.fl & 1u), by = PAD != PAD_ZEROS && (g.fl & 2u);
        const bool bz = PAD != PAD_ZEROS && (g.fl & 4u);
        const float gx0 = fmaf(g.ay, e01 - e00, e00), gx1 = fmaf(g.ay, e11 - e10, e10);
        t.dx = bx ? 0.0f : fmaf(g.az, gx1 - gx0, gx0);
        t.dy = by ? 0.0f : fmaf(g.az, f1 - f0, f0);
        t.dz = bz ? 0.0f : (c1 - c0);
    } else {
        t.dx = t.dy = t.dz = 0.0f;
    }
    return t;
}

// Software pipeline of one thread's walk down its (x, y) column over
// [z0, z1): the corners of z+1 are gathered while z is processed, and u of
// z+2 is loaded meanwhile.  Two register sets alternate with the slice's
// parity (S = (z - z0) & 1), and the kernels take two slices per loop
// iteration (step<0> then step<1>), so pending registers are never copied:
// a copy (what the compiler emits for a loop-carried load destination
// written under a branch, or reused across iterations) waits for the loads
// just issued and undoes the pipeline.
template <int PAD, bool AFF>
struct ColumnSampler {
    const MiArgs& a;
    int x, y, HW, z1;
    size_t N;
    MiPend p[2];
    float un[2][3];

    __device__ ColumnSampler(const MiArgs& a_, int x_, int y_, int z0, int z1_)
        : a(a_), x(x_), y(y_), HW(a_.H * a_.W), z1(z1_), N((size_t)a_.D * a_.H * a_.W)
    {
        if (z0 >= z1) return;  // empty column: no loads
        float u0[3];
        load_u(z0, u0);
        issue(z0, u0, p[0]);
        load_u(min(z0 + 1, z1 - 1), un[1]);
    }
    __device__ void load_u(int zz, float* o)
    {
        const int id = zz * HW + y * a.W + x;
        if (a.u) {  // each element read once per kernel: non-temporal
            o[0] = __builtin_nontemporal_load(a.u + id);
            o[1] = __builtin_nontemporal_load(a.u + N + id);
            o[2] = __builtin_nontemporal_load(a.u + 2 * N + id);
        }
        else { o[0] = 0.f; o[1] = 0.f; o[2] = 0.f; }
    }
    __device__ void issue(int zz, const float* uu, MiPend& g)
    {
        float dx, dy, dz;
        if (AFF) affine_disp(a.aff, x, y, zz, uu[0], uu[1], uu[2], dx, dy, dz);
        else { dx = uu[0]; dy = uu[1]; dz = uu[2]; }
        mi_issue<PAD>(a, x, y, zz, dx, dy, dz, zz * HW + y * a.W + x, g);
    }
    // the loads of z (issued one step ago); issues those of z + 1 and u of
    // z + 2, clamped into the column (past its end they repeat the last
    // slice and are never used)
    template <int S>
    __device__ MiPend step(int z)
    {
        const MiPend cur = p[S];
        issue(min(z + 1, z1 - 1), un[1 - S], p[1 - S]);
        load_u(min(z + 2, z1 - 1), un[S]);
        return cur;
    }
};

// Row pitch of the LDS histogram copies: at least B + 5 columns (Mw bins -2 ..
// B + 1 of the Parzen window; the hard-bin patch j .. j + 3 of j <= B - 1
// reaches column B + 4), odd.
__host__ __device__ constexpr int mi_hist_pitch(int B) { return (B + 5) | 1; }

// GLOB: the histogram is too large for LDS (a.ncopy == 0) and the taps are
// added straight into the global one; otherwise into a.ncopy LDS copies.
// (Compile-time, so that each atomic is an LDS or a global one, never flat.)
template <bool HARD, int PAD, bool AFF, bool GLOB>
__global__ void __launch_bounds__(MI_NT) mi_hist_kernel(MiArgs a, unsigned long long* __restrict__ ghist,
                                                        unsigned long long* __restrict__ gflag)
{
    // LDS: a.ncopy copies of B rows (F bins, clamped) of mi_hist_pitch(B)
    // >= B + 5 columns holding the Mw bins -2 .. B + 1 unclamped (column c at
    // c + 2), so the four columns of a patch are consecutive and each row of
    // the flush is one address plus immediate offsets; the clamp of those
    // columns into bins 0 and B - 1 happens once, when the copies are added
    // up.  The pitch is odd: with an even one (a row is twice as many banks
    // wide) the same column of any two rows falls in one LDS bank, which is
    // what lanes with equal Mw bins and different F bins hit.  Copy stride
    // B pitch + 1.  GLOB: the global [B][B] histogram, columns clamped.
    extern __shared__ unsigned long long hist[];
    const int B = a.bins, BB = B * B;
    const int RP = GLOB ? B : mi_hist_pitch(B), CS = B * RP + 1;  // row pitch, copy stride
    for (int q = threadIdx.x; !GLOB && q < a.ncopy * CS; q += MI_NT) hist[q] = 0ull;
    unsigned long long* const mine = GLOB ? ghist : hist + (threadIdx.x & (a.ncopy - 1)) * CS;
    __shared__ int nanflag;
    if (threadIdx.x == 0) nanflag = 0;
    __syncthreads();

    const int bid = xcd_remap(blockIdx.x, a.nblocks);
    const int tx = bid % a.ntx, rest = bid / a.ntx, ty = rest % a.nty, ch = rest / a.nty;
    const int x = a.roi[4] + tx * MI_TX + (threadIdx.x % MI_TX);
    const int y = a.roi[2] + ty * MI_TY + (threadIdx.x / MI_TX);
    const int zb = a.roi[0] + ch * a.zchunk;
    const int ze = min(a.roi[1], zb + a.zchunk);
    const int H = a.H, W = a.W, HW = H * W;
    const size_t N = (size_t)a.D * HW;
    const bool active = x < a.roi[5] && y < a.roi[3];

    int cm = -1000, cn = -1000;  // current 4x4 patch origin (sentinel: none)
    float acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
    bool bad = false;

    auto flush = [&]() {
        if (GLOB) {
            int row[4], col[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                row[i] = (int)__umul24((unsigned)fold(cm + i, B), (unsigned)RP);
                col[i] = fold(cn + i, B);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    atomicAdd(&mine[row[i] + col[jj]], to_fix(acc[i * 4 + jj]));  // unconditional: no branch per tap
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                unsigned long long* rp = mine + (int)__umul24((unsigned)fold(cm + i, B), (unsigned)RP) + (cn + 2);
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) atomicAdd(rp + jj, to_fix(acc[i * 4 + jj]));
            }
        }
    };

    auto voxel = [&](const MiPend& sp) {
        const float fv = sp.f;
        const float mv = mi_interp<PAD, false>(sp).v;
        bad |= (fv != fv) || (mv != mv);
        int jf, jm;
        float wf[4], wm[4], dd[4];
        parzen4<HARD, false>(fv, B, jf, wf, dd);
        parzen4<HARD, false>(mv, B, jm, wm, dd);
        if (jf != cm || jm != cn) {
            if (cm != -1000) flush();
            cm = jf; cn = jm;
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) acc[i * 4 + jj] = fmaf(wf[i], wm[jj], acc[i * 4 + jj]);
    };
    if (active && zb < ze) {
        ColumnSampler<PAD, AFF> cs(a, x, y, zb, ze);
        for (int z = zb; z < ze; z += 2) {
            const MiPend s0 = cs.template step<0>(z);
            voxel(s0);
            const MiPend s1 = cs.template step<1>(z + 1);
            if (z + 1 < ze) voxel(s1);
        }
        if (cm != -1000) flush();
    }
    if (bad) nanflag = 1;
    __syncthreads();
    for (int q = threadIdx.x; !GLOB && q < BB; q += MI_NT) {
        const int r = q / B, c = q - r * B;
        // stored columns of bin c: c + 2, and the clamped ones beside the edges
        const int s0 = c == 0 ? 0 : c + 2, s1 = c == B - 1 ? B + 3 : c + 2;
        unsigned long long v = 0ull;
        for (int k = 0; k < a.ncopy; ++k)
            for (int sc = s0; sc <= s1; ++sc) v += hist[k * CS + r * RP + sc];
        if (v) atomicAdd(&ghist[q], v);
    }
    if (threadIdx.x == 0 && nanflag) atomicOr(gflag, 1ull);
}

template <int PAD, bool AFF>
__global__ void __launch_bounds__(MI_NT) mi_count_kernel(MiArgs a, unsigned long long* __restrict__ ghist,
                                                         unsigned long long* __restrict__ gflag)
{
    extern __shared__ unsigned int cnt[];  // a.ncopy copies of [B*B], stride B*B+1
    const int B = a.bins, BB = B * B, CS = BB + 1;
    for (int q = threadIdx.x; q < a.ncopy * CS; q += MI_NT) cnt[q] = 0u;
    unsigned int* const mine = cnt + (threadIdx.x & (a.ncopy > 0 ? a.ncopy - 1 : 0)) * CS;
    const bool glob = a.ncopy == 0;  // counts too large for LDS: add straight into the global histogram
    __shared__ int nanflag;
    if (threadIdx.x == 0) nanflag = 0;
    __syncthreads();

    const int bid = xcd_remap(blockIdx.x, a.nblocks);
    const int tx = bid % a.ntx, rest = bid / a.ntx, ty = rest % a.nty, ch = rest / a.nty;
    const int x = a.roi[4] + tx * MI_TX + (threadIdx.x % MI_TX);
    const int y = a.roi[2] + ty * MI_TY + (threadIdx.x / MI_TX);
    const int zb = a.roi[0] + ch * a.zchunk;
    const int ze = min(a.roi[1], zb + a.zchunk);
    const int H = a.H, W = a.W, HW = H * W;
    const size_t N = (size_t)a.D * HW;
    const bool active = x < a.roi[5] && y < a.roi[3];
    int cur = -1;
    unsigned run = 0u;
    bool bad = false;
    auto voxel = [&](const MiPend& sp) {
        const float fv = sp.f;
        const float mv = mi_interp<PAD, false>(sp).v;
        bad |= (fv != fv) || (mv != mv);
        const int bf = exact_bin(fminf(fmaxf(fv, 0.0f), 1.0f), B);
        const int bm = exact_bin(fminf(fmaxf(mv, 0.0f), 1.0f), B);
        const int q = bf * B + bm;
        if (q != cur) {
            if (run) {
                if (glob) atomicAdd(&ghist[cur], (unsigned long long)run);
                else atomicAdd(&mine[cur], run);
            }
            cur = q;
            run = 0u;
        }
        ++run;
    };
    if (active && zb < ze) {
        ColumnSampler<PAD, AFF> cs(a, x, y, zb, ze);
        for (int z = zb; z < ze; z += 2) {
            const MiPend s0 = cs.template step<0>(z);
            voxel(s0);
            const MiPend s1 = cs.template step<1>(z + 1);
            if (z + 1 < ze) voxel(s1);
        }
        if (run) {
            if (glob) atomicAdd(&ghist[cur], (unsigned long long)run);
            else atomicAdd(&mine[cur], run);
        }
    }
    if (bad) nanflag = 1;
    __syncthreads();
    for (int q = threadIdx.x; !glob && q < BB; q += MI_NT) {
        unsigned long long v = 0ull;
        for (int c = 0; c < a.ncopy; ++c) v += cnt[c * CS + q];
        if (v) atomicAdd(&ghist[q], v);
    }
    if (threadIdx.x == 0 && nanflag) atomicOr(gflag, 1ull);
}

// Weight that bin m receives from a sample at the centre of bin j (cubic
// B-spline taps 2/3 at the centre and 1/6 at distance one, folded at the
// edges like the soft kernel).
__device__ __forceinline__ double centre_tap(int m, int j, int B)
{
    double w = 0.0;
#pragma unroll
    for (int off = -1; off <= 1; ++off)
        if (fold(j + off, B) == m) w += off == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
    return w;
}

// Entry (m, n) of the approximate PMF p = K (counts / total) K^T.
__device__ __forceinline__ double approx_p(const unsigned long long* __restrict__ hist, int B, int m, int n,
                                          double sc)
{
    double acc = 0.0;
    for (int i = max(m - 1, 0); i <= min(m + 1, B - 1); ++i) {
        const double wi = centre_tap(m, i, B);
        if (wi == 0.0) continue;
        double row = 0.0;
        for (int j = max(n - 1, 0); j <= min(n + 1, B - 1); ++j) row += centre_tap(n, j, B) * (double)hist[i * B + j];
        acc += wi * row;
    }
    return acc * sc;
}

// One block: the approximate PMF p = K (counts / total) K^T, marginals, MI and
// the log table, with the same state layout as mi_finalize.  Entries of p
// are recomputed where needed (nine taps each) instead of held, so any
// B <= 256 fits.
__global__ void __launch_bounds__(1024) mi_finalize_approx(const unsigned long long* __restrict__ hist,
                                                           const unsigned long long* __restrict__ flag, int B,
                                                           float* __restrict__ state, float* __restrict__ loss)
{
    __shared__ double pF[MI_MAX_BINS], pM[MI_MAX_BINS];
    __shared__ unsigned long long rowsum[MI_MAX_BINS];
    __shared__ double red[1024];
    const int BB = B * B;
    for (int t = threadIdx.x; t < B; t += 1024) {
        unsigned long long rs = 0;
        for (int n = 0; n < B; ++n) rs += hist[t * B + n];
        rowsum[t] = rs;
    }
    __syncthreads();
    unsigned long long total = 0;
    for (int t = 0; t < B; ++t) total += rowsum[t];
    const double sc = total ? 1.0 / (double)total : 0.0;
    for (int t = threadIdx.x; t < B; t += 1024) {
        double rf = 0.0, cm = 0.0;
        for (int n = 0; n < B; ++n) { rf += approx_p(hist, B, t, n, sc); cm += approx_p(hist, B, n, t, sc); }
        pF[t] = rf;
        pM[t] = cm;
    }
    __syncthreads();
    double part = 0.0;
    for (int q = threadIdx.x; q < BB; q += 1024) {
        const int m = q / B, n = q - m * B;
        const double p = approx_p(hist, B, m, n, sc);
        float tv = 0.0f;
        if (p > 0.0) {
            part += p * log(p / (pF[m] * pM[n]));
            tv = (float)(log(p) - log(pM[n]));
        }
        state[q] = tv;
        state[BB + q] = (float)p;
    }
    for (int t = threadIdx.x; t < B; t += 1024) {
        state[2 * BB + t] = (float)pF[t];
        state[2 * BB + B + t] = (float)pM[t];
    }
    const double mi = block_sum<1024>(part, red);
    if (threadIdx.x == 0) {
        const float l = (*flag) ? __int_as_float(0x7fc00000) : (float)(-mi);
        float* hdr = state + 2 * BB + 2 * B;
        hdr[0] = l;
        hdr[1] = (float)mi;
        hdr[2] = (float)B;
        for (int k = 3; k < 16; ++k) hdr[k] = 0.0f;  // reserved
        *loss = l;
    }
}

__global__ void __launch_bounds__(256) mi_zero(unsigned long long* p, int n)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0ull;
}

// One block: p, marginals, MI, log table.  Fixed-order reductions.  The
// histogram is normalised by its own total (exact integer sum): the B-spline
// weights partition unity only up to fp32 rounding, and dividing by the total
// keeps p a probability mass function, so that for instance p = p_F p_M
// holds to the fixed-point resolution when it holds exactly.
__global__ void __launch_bounds__(1024) mi_finalize(const unsigned long long* __restrict__ hist,
                                                    const unsigned long long* __restrict__ flag, int B,
                                                    float* __restrict__ state, float* __restrict__ loss)
{
    __shared__ double pF[MI_MAX_BINS], pM[MI_MAX_BINS];
    __shared__ unsigned long long rowsum[MI_MAX_BINS];
    __shared__ double red[1024];
    const int BB = B * B;
    for (int t = threadIdx.x; t < B; t += 1024) {
        unsigned long long rs = 0;
        for (int n = 0; n < B; ++n) rs += hist[t * B + n];
        rowsum[t] = rs;
    }
    __syncthreads();
    unsigned long long total = 0;
    for (int t = 0; t < B; ++t) total += rowsum[t];
    const double sc = total ? 1.0 / (double)total : 0.0;
    for (int t = threadIdx.x; t < B; t += 1024) {
        unsigned long long cs = 0;
        for (int m = 0; m < B; ++m) cs += hist[m * B + t];
        pF[t] = (double)rowsum[t] * sc;
        pM[t] = (double)cs * sc;
    }
    __syncthreads();
    double part = 0.0;
    for (int q = threadIdx.x; q < BB; q += 1024) {
        const int m = q / B, n = q - m * B;
        const double p = (double)hist[q] * sc;
        float tv = 0.0f;
        if (p > 0.0) {
            part += p * log(p / (pF[m] * pM[n]));
            tv = (float)(log(p) - log(pM[n]));
        }
        state[q] = tv;
        state[BB + q] = (float)p;
    }
    for (int t = threadIdx.x; t < B; t += 1024) {
        state[2 * BB + t] = (float)pF[t];
        state[2 * BB + B + t] = (float)pM[t];
    }
    const double mi = block_sum<1024>(part, red);
    if (threadIdx.x == 0) {
        const float l = (*flag) ? __int_as_float(0x7fc00000) : (float)(-mi);
        float* hdr = state + 2 * BB + 2 * B;
        hdr[0] = l;
        hdr[1] = (float)mi;
        hdr[2] = (float)B;
        for (int k = 3; k < 16; ++k) hdr[k] = 0.0f;  // reserved
        *loss = l;
    }
}

// TP > 0: the log table is staged in LDS, padded (B <= MI_LDS_TABLE_BINS);
// TP = 0: larger tables are read from the state through the caches.
// (Compile-time, so the table reads are LDS or global loads, never flat.)
template <bool HARD, int PAD, bool AFF, int TP>
__global__ void __launch_bounds__(MI_NT) mi_grad_kernel(MiArgs a, const float* __restrict__ state,
                                                        const float* __restrict__ grad_scale, float neg_inv_nroi,
                                                        float* __restrict__ gu)
{
    // TP > 0: the log table in LDS with 2 entries of padding on every side
    // and row pitch TP >= B + 4, Tp[(m + 2) TP + n + 2] = T[fold(m)][fold(n)]
    // for m, n in [-2, B + 1], so that the 4 x 4 lookups of a voxel need no
    // folding and sit at compile-time offsets from one address.  TP = 0: T
    // read from global memory with folded indices.
    extern __shared__ float Ts[];  // [TP * TP] when TP > 0
    const int B = a.bins;
    for (int q = threadIdx.x; TP > 0 && q < TP * TP; q += MI_NT) {
        const int m = q / TP - 2, n = q % TP - 2;
        Ts[q] = (m < B + 2 && n < B + 2) ? state[fold(m, B) * B + fold(n, B)] : 0.0f;
    }
    __syncthreads();
    const float g = neg_inv_nroi * (grad_scale ? *grad_scale : 1.0f);

    const int bid = xcd_remap(blockIdx.x, a.nblocks);
    const int tx = bid % a.ntx, rest = bid / a.ntx, ty = rest % a.nty, ch = rest / a.nty;
    const int x = tx * MI_TX + (threadIdx.x % MI_TX);
    const int y = ty * MI_TY + (threadIdx.x / MI_TX);
    const int zb = ch * a.zchunk, ze = min(a.D, zb + a.zchunk);
    const int H = a.H, W = a.W, HW = H * W;
    const size_t N = (size_t)a.D * HW;
    const bool active = x < W && y < H;
    const bool colroi = active && x >= a.roi[4] && x < a.roi[5] && y >= a.roi[2] && y < a.roi[3];
    // Every lane samples: lanes past the array read a valid column and lanes
    // outside the ROI columns have their gradient zeroed, so the sampling
    // branches depend only on z (uniform over the block) and no lane skips
    // the pipelined loads (see ColumnSampler).
    const int xc = min(x, W - 1), yc = min(y, H - 1);
    double acc[AFF ? 12 : 1];
#pragma unroll
    for (int q = 0; q < (AFF ? 12 : 1); ++q) acc[q] = 0.0;
    const int zr0 = max(zb, a.roi[0]), zr1 = min(ze, a.roi[1]);  // ROI slices of this chunk
    const bool samp = !HARD && zr0 < zr1;
    const int s0 = samp ? zr0 : ze, s1 = samp ? zr1 : ze;      // sampled slices [s0, s1)
    auto store = [&](int z, float g0, float g1, float g2) {
        if (active && (!AFF || gu)) {
            const int idx = z * HW + y * W + x;  // written once, never read here
            __builtin_nontemporal_store(g0, gu + idx);
            __builtin_nontemporal_store(g1, gu + N + idx);
            __builtin_nontemporal_store(g2, gu + 2 * N + idx);
        }
    };
    auto voxel = [&](int z, const MiPend& cur) {
        const Tri t = mi_interp<PAD, true>(cur);
        int jf, jm;
        float wf[4], wm[4], dm[4], dd[4];
        parzen4<false, false>(cur.f, B, jf, wf, dd);
        parzen4<false, true>(t.v, B, jm, wm, dm);
        float S = 0.0f;
        if (TP > 0) {
            const float* base = Ts + (jf + 2) * TP + (jm + 2);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float si = 0.0f;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) si = fmaf(dm[jj], base[i * TP + jj], si);
                S = fmaf(wf[i], si, S);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float* row = state + fold(jf + i, B) * B;
                float si = 0.0f;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) si = fmaf(dm[jj], row[fold(jm + jj, B)], si);
                S = fmaf(wf[i], si, S);
            }
        }
        const float gm = colroi ? g * S : 0.0f;
        float g0 = gm * t.dx, g1 = gm * t.dy, g2 = gm * t.dz;
        if (AFF) affine_adjoint(a.aff, xc, yc, z, g0, g1, g2, acc, g0, g1, g2);
        store(z, g0, g1, g2);
    };
    for (int z = zb; z < s0; ++z) store(z, 0.f, 0.f, 0.f);
    if (s0 < s1) {
        ColumnSampler<PAD, AFF> cs(a, xc, yc, s0, s1);
        for (int z = s0; z < s1; z += 2) {
            const MiPend c0 = cs.template step<0>(z);
            voxel(z, c0);
            const MiPend c1 = cs.template step<1>(z + 1);
            if (z + 1 < s1) voxel(z + 1, c1);
        }
    }
    for (int z = s1; z < ze; ++z) store(z, 0.f, 0.f, 0.f);
    if (AFF) {
        __shared__ double red[MI_NT];
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            const double v = block_sum<MI_NT>(acc[AFF ? q : 0], red);
            if (threadIdx.x == 0) a.apart[12 * (size_t)blockIdx.x + q] = v;
        }
    }
}

MiLaunch mi_plan(int rz, int ry, int rx)
{
    MiLaunch L;
    L.ntx = (rx + MI_TX - 1) / MI_TX;
    L.nty = (ry + MI_TY - 1) / MI_TY;
    const int tiles = L.ntx * L.nty;
    int chunks = 4096 / tiles;
    const int maxchunks = (rz + 31) / 32;
    if (chunks > maxchunks) chunks = maxchunks;
    if (chunks < 1) chunks = 1;
    L.zchunk = (rz + chunks - 1) / chunks;
    L.nchunks = (rz + L.zchunk - 1) / L.zchunk;
    L.nblocks = tiles * L.nchunks;
    return L;
}

template <bool AFF>
static hipError_t mi_fwd_dispatch(const MiArgs& a, int hard, int pad, unsigned long long* hist,
                                  unsigned long long* flag, float* state, float* loss, hipStream_t st)
{
    const int BB = a.bins * a.bins;
    dim3 grid(a.nblocks), block(MI_NT);
    if (hard == 2) {
        const size_t lds32 = sizeof(unsigned int) * a.ncopy * (BB + 1);
        if (pad == PAD_BORDER) hipLaunchKernelGGL((mi_count_kernel<PAD_BORDER, AFF>), grid, block, lds32, st, a, hist, flag);
        else if (pad == MI_PAD_BORDER1) hipLaunchKernelGGL((mi_count_kernel<MI_PAD_BORDER1, AFF>), grid, block, lds32, st, a, hist, flag);
        else hipLaunchKernelGGL((mi_count_kernel<PAD_ZEROS, AFF>), grid, block, lds32, st, a, hist, flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(mi_finalize_approx, dim3(1), dim3(1024), 0, st, hist, flag, a.bins, state, loss);
        return hipGetLastError();
    }
    const size_t lds = sizeof(unsigned long long) * a.ncopy * (a.bins * mi_hist_pitch(a.bins) + 1);
    if (a.ncopy == 0) {
        if (hard) {
            if (pad == PAD_BORDER) hipLaunchKernelGGL((mi_hist_kernel<true, PAD_BORDER, AFF, true>), grid, block, 0, st, a, hist, flag);
            else if (pad == MI_PAD_BORDER1) hipLaunchKernelGGL((mi_hist_kernel<true, MI_PAD_BORDER1, AFF, true>), grid, block, 0, st, a, hist, flag);
            else hipLaunchKernelGGL((mi_hist_kernel<true, PAD_ZEROS, AFF, true>), grid, block, 0, st, a, hist, flag);
        } else {
            if (pad == PAD_BORDER) hipLaunchKernelGGL((mi_hist_kernel<false, PAD_BORDER, AFF, true>), grid, block, 0, st, a, hist, flag);
            else if (pad == MI_PAD_BORDER1) hipLaunchKernelGGL((mi_hist_kernel<false, MI_PAD_BORDER1, AFF, true>), grid, block, 0, st, a, hist, flag);
            else hipLaunchKernelGGL((mi_hist_kernel<false, PAD_ZEROS, AFF, true>), grid, block, 0, st, a, hist, flag);
        }
    } else if (hard) {
        if (pad == PAD_BORDER) hipLaunchKernelGGL((mi_hist_kernel<true, PAD_BORDER, AFF, false>), grid, block, lds, st, a, hist, flag);
        else if (pad == MI_PAD_BORDER1) hipLaunchKernelGGL((mi_hist_kernel<true, MI_PAD_BORDER1, AFF, false>), grid, block, lds, st, a, hist, flag);
        else hipLaunchKernelGGL((mi_hist_kernel<true, PAD_ZEROS, AFF, false>), grid, block, lds, st, a, hist, flag);
    } else {
        if (pad == PAD_BORDER) hipLaunchKernelGGL((mi_hist_kernel<false, PAD_BORDER, AFF, false>), grid, block, lds, st, a, hist, flag);
        else if (pad == MI_PAD_BORDER1) hipLaunchKernelGGL((mi_hist_kernel<false, MI_PAD_BORDER1, AFF, false>), grid, block, lds, st, a, hist, flag);
        else hipLaunchKernelGGL((mi_hist_kernel<false, PAD_ZEROS, AFF, false>), grid, block, lds, st, a, hist, flag);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mi_finalize, dim3(1), dim3(1024), 0, st, hist, flag, a.bins, state, loss);
    return hipGetLastError();
}

hipError_t mi_fwd_launch(const MiArgs& a0, int hard, int pad, unsigned long long* hist, float* state, float* loss,
                         double nroi, hipStream_t st)
{
    (void)nroi;
    MiArgs a = a0;
    // LDS histogram copies: at most 4 and at most 79 KB (two blocks per CU).
    // u64 for the Parzen histogram, rows of mi_hist_pitch(B) entries: 4
    // copies up to 47 bins, 2 up to 68, 1 up to 98; u32 counts of the
    // approximate estimator within 66 KB: 1 copy up to 128 bins.  Larger
    // histograms are added straight into the global one (ncopy = 0).
    const size_t budget = hard == 2 ? 67584 : 80896;
    const size_t one = hard == 2 ? (size_t)(a.bins * a.bins + 1) * sizeof(unsigned int)
                                 : (size_t)(a.bins * mi_hist_pitch(a.bins) + 1) * sizeof(unsigned long long);
    a.ncopy = one <= budget ? 1 : 0;
    while (a.ncopy && a.ncopy < 4 && 2 * a.ncopy * one <= budget) a.ncopy *= 2;
    const int BB = a.bins * a.bins;
    unsigned long long* flag = hist + BB;
    hipLaunchKernelGGL(mi_zero, dim3((BB + 1 + 255) / 256), dim3(256), 0, st, hist, BB + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int p = (pad == PAD_BORDER && a.W < 2) ? MI_PAD_BORDER1 : pad;
    return a.affine ? mi_fwd_dispatch<true>(a, hard, p, hist, flag, state, loss, st)
                    : mi_fwd_dispatch<false>(a, hard, p, hist, flag, state, loss, st);
}

template <bool HARD, bool AFF, int TP>
static void mi_grad_launch_pad(int pad, dim3 grid, size_t lds, hipStream_t st, const MiArgs& a, const float* state,
                               const float* grad_scale, float nin, float* gu)
{
    if (pad == PAD_BORDER)
        hipLaunchKernelGGL((mi_grad_kernel<HARD, PAD_BORDER, AFF, TP>), grid, dim3(MI_NT), lds, st, a, state, grad_scale, nin, gu);
    else if (pad == MI_PAD_BORDER1)
        hipLaunchKernelGGL((mi_grad_kernel<HARD, MI_PAD_BORDER1, AFF, TP>), grid, dim3(MI_NT), lds, st, a, state, grad_scale, nin, gu);
    else
        hipLaunchKernelGGL((mi_grad_kernel<HARD, PAD_ZEROS, AFF, TP>), grid, dim3(MI_NT), lds, st, a, state, grad_scale, nin, gu);
}

// The padded LDS table pitch: the smallest of 36, 68, 132 that holds B + 4
// columns (B <= 128); larger tables are read from global memory.
template <bool AFF>
static hipError_t mi_bwd_dispatch(const MiArgs& a, int hard, int pad, const float* state, const float* grad_scale,
                                  float nin, float* gu, hipStream_t st)
{
    const int B = a.bins;
    const dim3 grid(a.nblocks);
    if (hard == 1)  // box kernel: zero gradient, the table is not read
        mi_grad_launch_pad<true, AFF, 0>(pad, grid, 0, st, a, state, grad_scale, nin, gu);
    else if (B + 4 <= 36)
        mi_grad_launch_pad<false, AFF, 36>(pad, grid, sizeof(float) * 36 * 36, st, a, state, grad_scale, nin, gu);
    else if (B + 4 <= 68)
        mi_grad_launch_pad<false, AFF, 68>(pad, grid, sizeof(float) * 68 * 68, st, a, state, grad_scale, nin, gu);
    else if (B <= MI_LDS_TABLE_BINS)
        mi_grad_launch_pad<false, AFF, 132>(pad, grid, sizeof(float) * 132 * 132, st, a, state, grad_scale, nin, gu);
    else
        mi_grad_launch_pad<false, AFF, 0>(pad, grid, 0, st, a, state, grad_scale, nin, gu);
    return hipGetLastError();
}

hipError_t mi_bwd_launch(const MiArgs& a, int hard, int pad, const float* state, const float* grad_scale,
                         float* gu, double nroi, hipStream_t st)
{
    const float nin = (float)(-1.0 / nroi);
    const int p = (pad == PAD_BORDER && a.W < 2) ? MI_PAD_BORDER1 : pad;
    return a.affine ? mi_bwd_dispatch<true>(a, hard, p, state, grad_scale, nin, gu, st)
                    : mi_bwd_dispatch<false>(a, hard, p, state, grad_scale, nin, gu, st);
}

}  // namespace ffdp
