// Device helpers shared by the HIP kernels: the implicit trilinear sampler,
// block-index remapping and reductions.  gfx950 (CDNA4), wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffdp {

enum { PAD_BORDER = 0, PAD_ZEROS = 1 };

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remap so that consecutive logical tiles (which share halo data) run on the
// same XCD: XCD x = b % 8 receives the blocks b = x, x + 8, ..., and takes
// the contiguous logical range that starts at x * (nb / 8) + min(x, nb % 8)
// (the first nb % 8 XCDs hold one block more).  A bijection of [0, nb) for
// every nb.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, rem = nb & 7, x = b & 7;
    return x * q + min(x, rem) + (b >> 3);
}

// One axis of the sample point p = x + u, split without forming x + u in
// fp32 (which would move the integer decision by an ulp of x): i0 = x +
// floor(u), alpha = u - floor(u).  Border mode clamps p to [0, n-1] and marks
// the axis clamped (zero derivative), also for a point exactly on the border.
template <int PAD>
__device__ __forceinline__ void axis_split(int x, float u, int n, int& i0, int& i1, float& a, bool& clamped)
{
    float f = floorf(u);
    // keep the index finite for huge or NaN displacements (NaN stays in `a`)
    f = fminf(fmaxf(f, -268435456.0f), 268435456.0f);
    a = u - f;
    i0 = x + (int)f;
    clamped = false;
    if (PAD == PAD_BORDER) {
        if (i0 < 0 || (i0 == 0 && a == 0.0f)) {
            i0 = 0; a = 0.0f; clamped = true;
        } else if (i0 >= n - 1) {
            i0 = n - 1; a = 0.0f; clamped = true;
        }
        i1 = min(i0 + 1, n - 1);
    } else {
        i1 = i0 + 1;
    }
}

struct Tri {
    float v, dx, dy, dz;
};

// Trilinear value of M at (x,y,z) + (ux,uy,uz) and, with DERIV, dvalue/dp.
template <int PAD, bool DERIV>
__device__ __forceinline__ Tri trilinear(const float* __restrict__ M, int D, int H, int W, int x, int y, int z,
                                         float ux, float uy, float uz)
{
    int x0, x1, y0, y1, z0, z1;
    float ax, ay, az;
    bool cx, cy, cz;
    axis_split<PAD>(x, ux, W, x0, x1, ax, cx);
    axis_split<PAD>(y, uy, H, y0, y1, ay, cy);
    axis_split<PAD>(z, uz, D, z0, z1, az, cz);
    float m000, m001, m010, m011, m100, m101, m110, m111;
    if (PAD == PAD_BORDER) {
        const int r00 = (z0 * H + y0) * W, r01 = (z0 * H + y1) * W;
        const int r10 = (z1 * H + y0) * W, r11 = (z1 * H + y1) * W;
        m000 = M[r00 + x0]; m001 = M[r00 + x1];
        m010 = M[r01 + x0]; m011 = M[r01 + x1];
        m100 = M[r10 + x0]; m101 = M[r10 + x1];
        m110 = M[r11 + x0]; m111 = M[r11 + x1];
    } else {
        const bool vx0 = (unsigned)x0 < (unsigned)W, vx1 = (unsigned)x1 < (unsigned)W;
        const bool vy0 = (unsigned)y0 < (unsigned)H, vy1 = (unsigned)y1 < (unsigned)H;
        const bool vz0 = (unsigned)z0 < (unsigned)D, vz1 = (unsigned)z1 < (unsigned)D;
        const int r00 = (z0 * H + y0) * W, r01 = (z0 * H + y1) * W;
        const int r10 = (z1 * H + y0) * W, r11 = (z1 * H + y1) * W;
        m000 = (vz0 && vy0 && vx0) ? M[r00 + x0] : 0.0f;
        m001 = (vz0 && vy0 && vx1) ? M[r00 + x1] : 0.0f;
        m010 = (vz0 && vy1 && vx0) ? M[r01 + x0] : 0.0f;
        m011 = (vz0 && vy1 && vx1) ? M[r01 + x1] : 0.0f;
        m100 = (vz1 && vy0 && vx0) ? M[r10 + x0] : 0.0f;
        m101 = (vz1 && vy0 && vx1) ? M[r10 + x1] : 0.0f;
        m110 = (vz1 && vy1 && vx0) ? M[r11 + x0] : 0.0f;
        m111 = (vz1 && vy1 && vx1) ? M[r11 + x1] : 0.0f;
    }
    // differences along x, then interpolate in x, y, z
    const float e00 = m001 - m000, e01 = m011 - m010, e10 = m101 - m100, e11 = m111 - m110;
    const float c00 = fmaf(ax, e00, m000), c01 = fmaf(ax, e01, m010);
    const float c10 = fmaf(ax, e10, m100), c11 = fmaf(ax, e11, m110);
    const float f0 = c01 - c00, f1 = c11 - c10;
    const float c0 = fmaf(ay, f0, c00), c1 = fmaf(ay, f1, c10);
    Tri t;
    t.v = fmaf(az, c1 - c0, c0);
    if (DERIV) {
        const float gx0 = fmaf(ay, e01 - e00, e00), gx1 = fmaf(ay, e11 - e10, e10);
        t.dx = cx ? 0.0f : fmaf(az, gx1 - gx0, gx0);
        t.dy = cy ? 0.0f : fmaf(az, f1 - f0, f0);
        t.dz = cz ? 0.0f : (c1 - c0);
    } else {
        t.dx = t.dy = t.dz = 0.0f;
    }
    return t;
}

// Border-mode trilinear sample with clamped corner indices, the form the
// streaming kernels use.  Along an axis whose sample point is clamped both
// corner indices coincide, so the value needs no special case and the corner
// difference (the derivative) is exactly zero; a point exactly on index 0 is
// also treated as clamped for the derivative.  Same results as
// trilinear<PAD_BORDER>.  Loads use 32-bit byte offsets from the volume base
// unless BIG (volumes of 2^30 voxels or more).
template <bool DERIV, bool BIG>
__device__ __forceinline__ Tri trilinear_clamped(const float* __restrict__ M, int D, int H, int W, int HW, int x,
                                                 int y, int z, float ux, float uy, float uz)
{
    const float fx = fminf(fmaxf(floorf(ux), -268435456.0f), 268435456.0f);
    const float fy = fminf(fmaxf(floorf(uy), -268435456.0f), 268435456.0f);
    const float fz = fminf(fmaxf(floorf(uz), -268435456.0f), 268435456.0f);
    const float ax = ux - fx, ay = uy - fy, az = uz - fz;
    const int ix = x + (int)fx, iy = y + (int)fy, iz = z + (int)fz;
    const int x0 = min(max(ix, 0), W - 1), x1 = min(max(ix + 1, 0), W - 1);
    const int y0 = min(max(iy, 0), H - 1), y1 = min(max(iy + 1, 0), H - 1);
    const int z0 = min(max(iz, 0), D - 1), z1 = min(max(iz + 1, 0), D - 1);
    float m000, m001, m010, m011, m100, m101, m110, m111;
    if (BIG) {
        const size_t r00 = (size_t)z0 * HW + (size_t)y0 * W, r01 = (size_t)z0 * HW + (size_t)y1 * W;
        const size_t r10 = (size_t)z1 * HW + (size_t)y0 * W, r11 = (size_t)z1 * HW + (size_t)y1 * W;
        m000 = M[r00 + x0]; m001 = M[r00 + x1]; m010 = M[r01 + x0]; m011 = M[r01 + x1];
        m100 = M[r10 + x0]; m101 = M[r10 + x1]; m110 = M[r11 + x0]; m111 = M[r11 + x1];
    } else {
        const char* base = reinterpret_cast<const char*>(M);
        const unsigned r00 = (unsigned)(z0 * HW + y0 * W) * 4u, r01 = (unsigned)(z0 * HW + y1 * W) * 4u;
        const unsigned r10 = (unsigned)(z1 * HW + y0 * W) * 4u, r11 = (unsigned)(z1 * HW + y1 * W) * 4u;
        const unsigned c0 = (unsigned)x0 * 4u, c1 = (unsigned)x1 * 4u;
        m000 = *reinterpret_cast<const float*>(base + (r00 + c0));
        m001 = *reinterpret_cast<const float*>(base + (r00 + c1));
        m010 = *reinterpret_cast<const float*>(base + (r01 + c0));
        m011 = *reinterpret_cast<const float*>(base + (r01 + c1));
        m100 = *reinterpret_cast<const float*>(base + (r10 + c0));
        m101 = *reinterpret_cast<const float*>(base + (r10 + c1));
        m110 = *reinterpret_cast<const float*>(base + (r11 + c0));
        m111 = *reinterpret_cast<const float*>(base + (r11 + c1));
    }
    const float e00 = m001 - m000, e01 = m011 - m010, e10 = m101 - m100, e11 = m111 - m110;
    const float c00 = fmaf(ax, e00, m000), c01 = fmaf(ax, e01, m010);
    const float c10 = fmaf(ax, e10, m100), c11 = fmaf(ax, e11, m110);
    const float f0 = c01 - c00, f1 = c11 - c10;
    const float c0 = fmaf(ay, f0, c00), c1 = fmaf(ay, f1, c10);
    Tri t;
    t.v = fmaf(az, c1 - c0, c0);
    if (DERIV) {
        const float gx0 = fmaf(ay, e01 - e00, e00), gx1 = fmaf(ay, e11 - e10, e10);
        t.dx = (ix == 0 && ax == 0.0f) ? 0.0f : fmaf(az, gx1 - gx0, gx0);
        t.dy = (iy == 0 && ay == 0.0f) ? 0.0f : fmaf(az, f1 - f0, f0);
        t.dz = (iz == 0 && az == 0.0f) ? 0.0f : (c1 - c0);
    } else {
        t.dx = t.dy = t.dz = 0.0f;
    }
    return t;
}

// Deterministic block sum of a double (fixed tree order).  All threads of the
// block must call it; `red` holds blockDim.x doubles of LDS.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red)
{
    // a tree over the largest power of two P <= NT; with NT not a power of
    // two, threads P .. NT - 1 first add into 0 .. NT - P - 1
    constexpr int P = (NT & (NT - 1)) == 0 ? NT : (NT >= 1024 ? 1024 : (NT >= 512 ? 512 : (NT >= 256 ? 256 : 128)));
    static_assert(P <= NT && 2 * P > NT && NT <= 2048, "block size");
    red[threadIdx.x] = v;
    __syncthreads();
    if (P < NT) {
        if ((int)threadIdx.x < NT - P) red[threadIdx.x] += red[threadIdx.x + P];
        __syncthreads();
    }
#pragma unroll
    for (int s = P / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

}  // namespace ffdp
