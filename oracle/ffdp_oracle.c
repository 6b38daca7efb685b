/*
 * FP64 CPU oracle for the fused warp + dissimilarity path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
 * link, load or call this file; only the tests, the smoke check and the CPU
 * timing leg of the benchmark do.  It shares no code with the HIP path.
 *
 * Every routine is the plain definition written out, in double precision,
 * with no blocking, fusion or reordering: inputs arrive as fp32 and are
 * converted exactly to double.  Each function names the passage it follows.
 *
 * Conventions:
 *   volumes  [D][H][W] C-order;  displacement u [3][D][H][W], channel 0 adds
 *   to x (W axis), 1 to y (H), 2 to z (D)  (App. "Composite Implicit Grid
 *   Sampler", Alg. gridsampler: X = (x,y,z), displacement u[:, z, y, x]).
 *   roi = {z0,z1,y0,y1,x0,x1}, half-open, or NULL for the whole array.
 *   pad: 0 = border (clamp), 1 = zeros.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef int64_t i64;

#define AT(z, y, x) ((((z) * H) + (y)) * W + (x))

static void roi_or_full(const i64* roi, i64 D, i64 H, i64 W, i64 r[6])
{
    if (roi) { memcpy(r, roi, 6 * sizeof(i64)); }
    else { r[0] = 0; r[1] = D; r[2] = 0; r[3] = H; r[4] = 0; r[5] = W; }
}

/* ------------------------------------------------------------------------ */
/* O1. Trilinear sample of M at p = x + u(x)                                 */
/* eq. (interp) of App. "Ring Sampler": the value is the sum over the eight  */
/* lattice neighbours of M times the product of 1-D hat weights.  Border     */
/* mode clamps p to [0, n-1] per axis and the derivative along a clamped     */
/* axis is zero; a point exactly on the border counts as clamped.  Zero mode */
/* treats lattice points outside the array as 0 (Alg. gridsampler).          */
/* ------------------------------------------------------------------------ */
static double sample_point(const float* M, i64 D, i64 H, i64 W, const double p[3] /* x,y,z */,
                           int pad, double dvdp[3] /* x,y,z; nullable */)
{
    const i64 n[3] = {W, H, D};
    double q[3];
    int clamped[3];
    for (int k = 0; k < 3; ++k) {
        q[k] = p[k];
        clamped[k] = 0;
        if (pad == 0) {
            if (q[k] <= 0.0) { q[k] = 0.0; clamped[k] = 1; }
            else if (q[k] >= (double)(n[k] - 1)) { q[k] = (double)(n[k] - 1); clamped[k] = 1; }
        }
    }
    i64 i0[3];
    double a[3];
    for (int k = 0; k < 3; ++k) { double f = floor(q[k]); i0[k] = (i64)f; a[k] = q[k] - f; }
    double val = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int bz = 0; bz < 2; ++bz)
        for (int by = 0; by < 2; ++by)
            for (int bx = 0; bx < 2; ++bx) {
                i64 cx = i0[0] + bx, cy = i0[1] + by, cz = i0[2] + bz;
                double m;
                if (cx < 0 || cx >= W || cy < 0 || cy >= H || cz < 0 || cz >= D) {
                    if (pad == 0) {  /* only reached with zero weight at the clamped edge */
                        cx = cx < 0 ? 0 : (cx >= W ? W - 1 : cx);
                        cy = cy < 0 ? 0 : (cy >= H ? H - 1 : cy);
                        cz = cz < 0 ? 0 : (cz >= D ? D - 1 : cz);
                        m = (double)M[AT(cz, cy, cx)];
                    } else {
                        m = 0.0;
                    }
                } else {
                    m = (double)M[AT(cz, cy, cx)];
                }
                double wx = bx ? a[0] : 1.0 - a[0];
                double wy = by ? a[1] : 1.0 - a[1];
                double wz = bz ? a[2] : 1.0 - a[2];
                val += m * wx * wy * wz;
                g[0] += m * (bx ? 1.0 : -1.0) * wy * wz;
                g[1] += m * (by ? 1.0 : -1.0) * wx * wz;
                g[2] += m * (bz ? 1.0 : -1.0) * wx * wy;
            }
    if (dvdp)
        for (int k = 0; k < 3; ++k) dvdp[k] = clamped[k] ? 0.0 : g[k];
    return val;
}

/* Mw(x) = M(x + u(x)) over the whole array; dMw [3][N] = dMw/dp (x,y,z). */
int orc_warp(const float* M, const float* u, i64 D, i64 H, i64 W, int pad, double* out, double* dout)
{
    const i64 N = D * H * W;
#pragma omp parallel for schedule(static)
    for (i64 z = 0; z < D; ++z)
        for (i64 y = 0; y < H; ++y)
            for (i64 x = 0; x < W; ++x) {
                i64 k = AT(z, y, x);
                double p[3] = {(double)x, (double)y, (double)z};
                if (u) { p[0] += (double)u[k]; p[1] += (double)u[N + k]; p[2] += (double)u[2 * N + k]; }
                double dv[3];
                out[k] = sample_point(M, D, H, W, p, pad, dv);
                if (dout) { dout[k] = dv[0]; dout[N + k] = dv[1]; dout[2 * N + k] = dv[2]; }
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O2. LNCC window statistics, eq. (lncc-loss) and (lncc-a/b/c):             */
/*   mu_F, mu_M = windowed means; A, B, C = windowed (co)variances taken in  */
/*   their centred form; W is the uniform w^3 box with weights 1/w^3, values */
/*   outside the array are 0 (zero-padded convolution).                      */
/* Sub-volume access: vals are given on the box [o, o+e) of the full array.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double* F;  /* on the sub-box */
    const double* Mw;
    i64 o[3];         /* z, y, x origin of the sub-box in the full array */
    i64 e[3];         /* extents */
    i64 D, H, W;      /* full array */
} vol_view;

static inline int in_array(const vol_view* v, i64 z, i64 y, i64 x)
{
    return z >= 0 && z < v->D && y >= 0 && y < v->H && x >= 0 && x < v->W;
}
static inline i64 vidx(const vol_view* v, i64 z, i64 y, i64 x)
{
    return ((z - v->o[0]) * v->e[1] + (y - v->o[1])) * v->e[2] + (x - v->o[2]);
}

static void lncc_stats(const vol_view* v, i64 z, i64 y, i64 x, int r,
                       double* muF, double* muM, double* A, double* B, double* C)
{
    const double inv = 1.0 / (double)((2 * r + 1) * (2 * r + 1) * (2 * r + 1));
    double sF = 0, sM = 0;
    for (i64 dz = -r; dz <= r; ++dz)
        for (i64 dy = -r; dy <= r; ++dy)
            for (i64 dx = -r; dx <= r; ++dx) {
                i64 zz = z + dz, yy = y + dy, xx = x + dx;
                if (!in_array(v, zz, yy, xx)) continue;
                i64 k = vidx(v, zz, yy, xx);
                sF += v->F[k];
                sM += v->Mw[k];
            }
    double mf = sF * inv, mm = sM * inv;
    double a = 0, b = 0, c = 0;
    for (i64 dz = -r; dz <= r; ++dz)
        for (i64 dy = -r; dy <= r; ++dy)
            for (i64 dx = -r; dx <= r; ++dx) {
                i64 zz = z + dz, yy = y + dy, xx = x + dx;
                double f = 0.0, m = 0.0;  /* padded voxels are 0 */
                if (in_array(v, zz, yy, xx)) { i64 k = vidx(v, zz, yy, xx); f = v->F[k]; m = v->Mw[k]; }
                a += (f - mf) * (m - mm);
                b += (f - mf) * (f - mf);
                c += (m - mm) * (m - mm);
            }
    *muF = mf; *muM = mm; *A = a * inv; *B = b * inv; *C = c * inv;
}

static inline int in_roi(const i64 r[6], i64 z, i64 y, i64 x)
{
    return z >= r[0] && z < r[1] && y >= r[2] && y < r[3] && x >= r[4] && x < r[5];
}

/* LNCC loss of (F, Mw) over the ROI: 1 - mean n_i, n_i = A^2/(B C + eps)
 * (eq. lncc-loss; the "1 - mean" form is that of Alg. lncc). */
double orc_lncc_loss(const float* F, const double* Mw, i64 D, i64 H, i64 W, const i64* roi, int w, double eps)
{
    i64 R[6];
    roi_or_full(roi, D, H, W, R);
    const i64 N = D * H * W;
    double* Fd = (double*)malloc(sizeof(double) * N);
    for (i64 k = 0; k < N; ++k) Fd[k] = (double)F[k];
    vol_view v = {Fd, Mw, {0, 0, 0}, {D, H, W}, D, H, W};
    const int r = (w - 1) / 2;
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(dynamic, 1)
    for (i64 z = R[0]; z < R[1]; ++z)
        for (i64 y = R[2]; y < R[3]; ++y)
            for (i64 x = R[4]; x < R[5]; ++x) {
                double mf, mm, A, B, C;
                lncc_stats(&v, z, y, x, r, &mf, &mm, &A, &B, &C);
                s += A * A / (B * C + eps);
            }
    free(Fd);
    const double nroi = (double)((R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]));
    return 1.0 - s / nroi;
}

/* ------------------------------------------------------------------------ */
/* O3. Gradient of the LNCC loss with respect to Mw.                         */
/* Chain rule of App. "Efficient Backward Pass" (eq. gradientcc-first ...     */
/* finalccgradM) redone for the moving image with eps kept:                  */
/*   g_i = dL/dn_i = -1/N_roi on the ROI;  D_i = B_i C_i + eps               */
/*   dn_i/dMw_k = w_ik [ 2A_i/D_i (F_k - muF_i) - 2 A_i^2 B_i/D_i^2 (Mw_k - muM_i) ] */
/*   dL/dMw_k   = sum_{i in ROI, k in window(i)} g_i dn_i/dMw_k              */
/* ANTs approximation (App. "ANTs gradient approximation"): the window sum   */
/* over i is dropped and the factors of voxel k itself are used.             */
/* ------------------------------------------------------------------------ */
static double lncc_dloss_dmw_at(const vol_view* v, const i64 R[6], i64 z, i64 y, i64 x, int r, double eps,
                                int ants, double nroi)
{
    const double inv = 1.0 / (double)((2 * r + 1) * (2 * r + 1) * (2 * r + 1));
    const double g = -1.0 / nroi;
    const i64 k = vidx(v, z, y, x);
    const double Fk = v->F[k], Mk = v->Mw[k];
    if (ants) {
        if (!in_roi(R, z, y, x)) return 0.0;
        double mf, mm, A, B, C;
        lncc_stats(v, z, y, x, r, &mf, &mm, &A, &B, &C);
        double Dn = B * C + eps;
        return g * (2.0 * A / Dn * (Fk - mf) - 2.0 * A * A * B / (Dn * Dn) * (Mk - mm));
    }
    double s = 0.0;
    for (i64 dz = -r; dz <= r; ++dz)
        for (i64 dy = -r; dy <= r; ++dy)
            for (i64 dx = -r; dx <= r; ++dx) {
                i64 zi = z + dz, yi = y + dy, xi = x + dx;
                if (!in_roi(R, zi, yi, xi)) continue;
                double mf, mm, A, B, C;
                lncc_stats(v, zi, yi, xi, r, &mf, &mm, &A, &B, &C);
                double Dn = B * C + eps;
                s += g * inv * (2.0 * A / Dn * (Fk - mf) - 2.0 * A * A * B / (Dn * Dn) * (Mk - mm));
            }
    return s;
}

/* Full LNCC oracle on (F, M, u): loss and, if grad_u != NULL, dL/du over the
 * whole array (dL/du_c = dL/dMw * dMw/dp_c, Alg. gridsampler Backward). */
int orc_lncc(const float* F, const float* M, const float* u, i64 D, i64 H, i64 W, const i64* roi,
             int w, double eps, int ants, int pad, double* loss, double* grad_u)
{
    const i64 N = D * H * W;
    i64 R[6];
    roi_or_full(roi, D, H, W, R);
    double* Mw = (double*)malloc(sizeof(double) * N);
    double* dM = grad_u ? (double*)malloc(sizeof(double) * 3 * N) : NULL;
    orc_warp(M, u, D, H, W, pad, Mw, dM);
    if (loss) *loss = orc_lncc_loss(F, Mw, D, H, W, R, w, eps);
    if (grad_u) {
        double* Fd = (double*)malloc(sizeof(double) * N);
        for (i64 k = 0; k < N; ++k) Fd[k] = (double)F[k];
        vol_view v = {Fd, Mw, {0, 0, 0}, {D, H, W}, D, H, W};
        const int r = (w - 1) / 2;
        const double nroi = (double)((R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]));
        /* the per-i factors of the chain rule are tabulated once, then the
         * sum over i in window(k) is taken for every k */
        double* a = (double*)calloc(N, sizeof(double));
        double* c = (double*)calloc(N, sizeof(double));
        double* mfa = (double*)calloc(N, sizeof(double));
        double* mmc = (double*)calloc(N, sizeof(double));
        const double g = -1.0 / nroi;
#pragma omp parallel for schedule(dynamic, 1)
        for (i64 z = R[0]; z < R[1]; ++z)
            for (i64 y = R[2]; y < R[3]; ++y)
                for (i64 x = R[4]; x < R[5]; ++x) {
                    double mf, mm, A, B, C;
                    lncc_stats(&v, z, y, x, r, &mf, &mm, &A, &B, &C);
                    double Dn = B * C + eps;
                    i64 i = AT(z, y, x);
                    a[i] = 2.0 * g * A / Dn;               /* factor of (F_k - muF_i) */
                    c[i] = 2.0 * g * A * A * B / (Dn * Dn); /* factor of (Mw_k - muM_i) */
                    mfa[i] = mf;
                    mmc[i] = mm;
                }
        const double inv = 1.0 / (double)((2 * r + 1) * (2 * r + 1) * (2 * r + 1));
#pragma omp parallel for schedule(dynamic, 1)
        for (i64 z = 0; z < D; ++z)
            for (i64 y = 0; y < H; ++y)
                for (i64 x = 0; x < W; ++x) {
                    i64 k = AT(z, y, x);
                    double s = 0.0;
                    if (ants) {
                        if (in_roi(R, z, y, x)) s = a[k] * (Fd[k] - mfa[k]) - c[k] * (Mw[k] - mmc[k]);
                    } else {
                        for (i64 dz = -r; dz <= r; ++dz)
                            for (i64 dy = -r; dy <= r; ++dy)
                                for (i64 dx = -r; dx <= r; ++dx) {
                                    i64 zi = z + dz, yi = y + dy, xi = x + dx;
                                    if (!in_roi(R, zi, yi, xi)) continue;
                                    i64 i = AT(zi, yi, xi);
                                    s += inv * (a[i] * (Fd[k] - mfa[i]) - c[i] * (Mw[k] - mmc[i]));
                                }
                    }
                    grad_u[k] = s * dM[k];
                    grad_u[N + k] = s * dM[N + k];
                    grad_u[2 * N + k] = s * dM[2 * N + k];
                }
        free(a); free(c); free(mfa); free(mmc); free(Fd);
    }
    free(Mw);
    if (dM) free(dM);
    return 0;
}

/* dL/du at selected voxels only (for arrays too large for the full oracle).
 * idx holds n triples (z, y, x); out receives n triples (d/du_x, d/du_y, d/du_z).
 * The ROI size, which sets g_i, is that of the whole array's ROI. */
int orc_lncc_grad_u_at(const float* F, const float* M, const float* u, i64 D, i64 H, i64 W, const i64* roi,
                       int w, double eps, int ants, int pad, const i64* idx, i64 n, double* out)
{
    i64 R[6];
    roi_or_full(roi, D, H, W, R);
    const int r = (w - 1) / 2;
    const i64 h = 2 * r;
    const i64 N = D * H * W;
    const double nroi = (double)((R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]));
#pragma omp parallel for schedule(dynamic, 1)
    for (i64 s = 0; s < n; ++s) {
        i64 z = idx[3 * s], y = idx[3 * s + 1], x = idx[3 * s + 2];
        i64 e = 2 * h + 1;
        double* Fl = (double*)malloc(sizeof(double) * e * e * e);
        double* Ml = (double*)malloc(sizeof(double) * e * e * e);
        vol_view v = {Fl, Ml, {z - h, y - h, x - h}, {e, e, e}, D, H, W};
        double dv_c[3] = {0, 0, 0};
        for (i64 zz = z - h; zz <= z + h; ++zz)
            for (i64 yy = y - h; yy <= y + h; ++yy)
                for (i64 xx = x - h; xx <= x + h; ++xx) {
                    i64 l = vidx(&v, zz, yy, xx);
                    if (!in_array(&v, zz, yy, xx)) { Fl[l] = 0.0; Ml[l] = 0.0; continue; }
                    i64 k = AT(zz, yy, xx);
                    double p[3] = {(double)xx, (double)yy, (double)zz};
                    if (u) { p[0] += (double)u[k]; p[1] += (double)u[N + k]; p[2] += (double)u[2 * N + k]; }
                    double dv[3];
                    Fl[l] = (double)F[k];
                    Ml[l] = sample_point(M, D, H, W, p, pad, dv);
                    if (zz == z && yy == y && xx == x) { dv_c[0] = dv[0]; dv_c[1] = dv[1]; dv_c[2] = dv[2]; }
                }
        double gm = lncc_dloss_dmw_at(&v, R, z, y, x, r, eps, ants, nroi);
        out[3 * s] = gm * dv_c[0];
        out[3 * s + 1] = gm * dv_c[1];
        out[3 * s + 2] = gm * dv_c[2];
        free(Fl); free(Ml);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O4. Parzen-window mutual information, eq. (mi) and App. "Vanilla MI".      */
/* Bin centres b_m = (m + 1/2)/B on [0,1]; kappa is the cubic B-spline in    */
/* units of the bin width, kappa_m(v) = beta3(s - m) with s = clamp(v,0,1) B  */
/* - 1/2.  Support falling outside [0, B-1] is folded onto the edge bin so   */
/* that sum_m kappa_m(v) = 1 for every v.  omega = d kappa / dv.             */
/* hard = 1: kappa_m(v) = 1[m = min(floor(v B), B-1)] (box kernel, omega = 0). */
/* hard = 2: the paper's approximate estimator (App. "Implicit MI", An        */
/* approximate histogram estimator): every sample counts once in its bin     */
/* min(floor(v B), B-1); the count histogram, divided by the sample count,   */
/* is convolved in both axes with kappa evaluated at bin-centre offsets,     */
/* K[m][m'] = kappa_m(b_m') (folded like kappa).  The gradient uses the      */
/* soft kernel's kappa and omega at the sample values with dL/dp taken at    */
/* the approximate p; where p[m][n] = 0, log p - log pM is taken as 0.       */
/* ------------------------------------------------------------------------ */
static double beta3(double t)
{
    double a = fabs(t);
    if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
    if (a < 2.0) { double q = 2.0 - a; return q * q * q / 6.0; }
    return 0.0;
}
static double dbeta3(double t)
{
    double a = fabs(t), sg = t < 0 ? -1.0 : 1.0;
    if (a < 1.0) return sg * (-12.0 * a + 9.0 * a * a) / 6.0;
    if (a < 2.0) { double q = 2.0 - a; return -sg * q * q / 2.0; }
    return 0.0;
}

/* Hard bin of a value already clamped to [0, 1]: m* = min(floor(v B), B-1)
 * (App. "Implicit MI implementation", approximate histogram estimator), with
 * v B and its floor taken in double on the value as given. */
static i64 hard_bin(double vc, int B)
{
    i64 m = (i64)floor(vc * (double)B);
    return m > B - 1 ? B - 1 : m;
}

/* kappa_m(v) and omega_m(v) for every m in [0, B). */
static void parzen_all(double v, int B, int hard, double* kap, double* om)
{
    for (int m = 0; m < B; ++m) { kap[m] = 0.0; om[m] = 0.0; }
    double vc = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    if (hard) {
        i64 m = hard_bin(vc, B);
        kap[m] = 1.0;
        return;
    }
    const double dsdv = (v >= 0.0 && v <= 1.0) ? (double)B : 0.0;
    const double s = vc * B - 0.5;
    /* every integer j with |s - j| < 2 contributes to bin clamp(j, 0, B-1) */
    for (i64 j = (i64)floor(s) - 2; j <= (i64)floor(s) + 2; ++j) {
        double t = s - (double)j;
        if (fabs(t) >= 2.0) continue;
        i64 m = j < 0 ? 0 : (j > B - 1 ? B - 1 : j);
        kap[m] += beta3(t);
        om[m] += dbeta3(t) * dsdv;
    }
}

/* MI of (F, Mw) over the ROI for an already warped Mw; loss = -MI.  p [B][B]
 * (row: F bin m, column: Mw bin n) receives the joint PMF if non-NULL.  If
 * dldmw != NULL it gets dloss/dMw over the whole array (zero outside the ROI):
 *   dMI/dp[m][n] = ln p[m][n] - ln pF[m] - ln pM[n] - 1   (marginals as sums)
 *   dp[m][n]/dMw_k = kappa_m(F_k) omega_n(Mw_k) / N_roi                     */
static int mi_core(const float* F, const double* Mw, i64 D, i64 H, i64 W, const i64* roi, int B, int hard,
                   double* loss, double* p_out, double* dldmw)
{
    i64 R[6];
    roi_or_full(roi, D, H, W, R);
    const double nroi = (double)((R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]));
    double* p = (double*)calloc((size_t)B * B, sizeof(double));
    const int approx = hard == 2;
    if (approx) hard = 0; /* soft kernel for the gradient */
    if (approx) {
        double* cnt = (double*)calloc((size_t)B * B, sizeof(double));
        for (i64 z = R[0]; z < R[1]; ++z)
            for (i64 y = R[2]; y < R[3]; ++y)
                for (i64 x = R[4]; x < R[5]; ++x) {
                    i64 k = AT(z, y, x);
                    double vf = (double)F[k], vm = Mw[k];
                    vf = vf < 0.0 ? 0.0 : (vf > 1.0 ? 1.0 : vf);
                    vm = vm < 0.0 ? 0.0 : (vm > 1.0 ? 1.0 : vm);
                    cnt[hard_bin(vf, B) * B + hard_bin(vm, B)] += 1.0;
                }
        /* K[m][j] = kappa_m(b_j), then p = K (cnt / N) K^T */
        double* K = (double*)malloc(sizeof(double) * B * B);
        double* kc = (double*)malloc(sizeof(double) * B);
        double* oc = (double*)malloc(sizeof(double) * B);
        for (int j = 0; j < B; ++j) {
            parzen_all(((double)j + 0.5) / (double)B, B, 0, kc, oc);
            for (int m = 0; m < B; ++m) K[m * B + j] = kc[m];
        }
        for (int m = 0; m < B; ++m)
            for (int nn = 0; nn < B; ++nn) {
                double acc = 0.0;
                for (int a = 0; a < B; ++a)
                    for (int b = 0; b < B; ++b) acc += K[m * B + a] * K[nn * B + b] * cnt[a * B + b];
                p[m * B + nn] = acc;
            }
        free(cnt); free(K); free(kc); free(oc);
    } else {
#pragma omp parallel
    {
        double* pl = (double*)calloc((size_t)B * B, sizeof(double));
        double* kf = (double*)malloc(sizeof(double) * B);
        double* km = (double*)malloc(sizeof(double) * B);
        double* of = (double*)malloc(sizeof(double) * B);
        double* om = (double*)malloc(sizeof(double) * B);
#pragma omp for schedule(static)
        for (i64 z = R[0]; z < R[1]; ++z)
            for (i64 y = R[2]; y < R[3]; ++y)
                for (i64 x = R[4]; x < R[5]; ++x) {
                    i64 k = AT(z, y, x);
                    parzen_all((double)F[k], B, hard, kf, of);
                    parzen_all(Mw[k], B, hard, km, om);
                    for (int m = 0; m < B; ++m) {
                        if (kf[m] == 0.0) continue;
                        for (int nn = 0; nn < B; ++nn) pl[m * B + nn] += kf[m] * km[nn];
                    }
                }
#pragma omp critical
        for (int q = 0; q < B * B; ++q) p[q] += pl[q];
        free(pl); free(kf); free(km); free(of); free(om);
    }
    }
    for (int q = 0; q < B * B; ++q) p[q] /= nroi;
    double* pF = (double*)calloc(B, sizeof(double));
    double* pM = (double*)calloc(B, sizeof(double));
    for (int m = 0; m < B; ++m)
        for (int nn = 0; nn < B; ++nn) { pF[m] += p[m * B + nn]; pM[nn] += p[m * B + nn]; }
    double mi = 0.0;
    for (int m = 0; m < B; ++m)
        for (int nn = 0; nn < B; ++nn) {
            double q = p[m * B + nn];
            if (q > 0.0) mi += q * log(q / (pF[m] * pM[nn]));
        }
    if (loss) *loss = -mi;
    if (p_out) memcpy(p_out, p, sizeof(double) * B * B);
    if (dldmw) {
#pragma omp parallel
        {
            double* kf = (double*)malloc(sizeof(double) * B);
            double* km = (double*)malloc(sizeof(double) * B);
            double* of = (double*)malloc(sizeof(double) * B);
            double* om = (double*)malloc(sizeof(double) * B);
#pragma omp for schedule(static)
            for (i64 z = 0; z < D; ++z)
                for (i64 y = 0; y < H; ++y)
                    for (i64 x = 0; x < W; ++x) {
                        i64 k = AT(z, y, x);
                        double s = 0.0;
                        if (in_roi(R, z, y, x)) {
                            parzen_all((double)F[k], B, hard, kf, of);
                            parzen_all(Mw[k], B, hard, km, om);
                            for (int m = 0; m < B; ++m)
                                for (int nn = 0; nn < B; ++nn) {
                                    double wgt = kf[m] * om[nn];
                                    if (wgt == 0.0) continue;
                                    const double q = p[m * B + nn];
                                    const double t = q > 0.0 ? log(q) - log(pM[nn]) : 0.0;
                                    double dmi = t - log(pF[m]) - 1.0;
                                    s += -wgt / nroi * dmi;
                                }
                        }
                        dldmw[k] = s;
                    }
            free(kf); free(km); free(of); free(om);
        }
    }
    free(p); free(pF); free(pM);
    return 0;
}


int orc_mi(const float* F, const float* M, const float* u, i64 D, i64 H, i64 W, const i64* roi,
           int B, int hard, int pad, double* loss, double* p_out, double* grad_u)
{
    const i64 N = D * H * W;
    double* Mw = (double*)malloc(sizeof(double) * N);
    double* dM = grad_u ? (double*)malloc(sizeof(double) * 3 * N) : NULL;
    double* s = grad_u ? (double*)malloc(sizeof(double) * N) : NULL;
    orc_warp(M, u, D, H, W, pad, Mw, dM);
    mi_core(F, Mw, D, H, W, roi, B, hard, loss, p_out, s);
    if (grad_u)
        for (i64 k = 0; k < N; ++k) {
            grad_u[k] = s[k] * dM[k];
            grad_u[N + k] = s[k] * dM[N + k];
            grad_u[2 * N + k] = s[k] * dM[2 * N + k];
        }
    free(Mw);
    if (dM) free(dM);
    if (s) free(s);
    return 0;
}

/* The same joint PMF for volumes too large to warp whole: each ROI voxel is
 * sampled (O1) and binned (O4) on the fly, with per-thread histograms added
 * at the end (the sums of mi_core in another order).  hard = 2 counts the
 * hard bins first and convolves with K as mi_core does.  n_edge (nullable)
 * receives the number of ROI voxels whose warped value, clamped to [0, 1],
 * lies within edge_tol of an interior bin edge m / B (0 < m < B), the
 * voxels whose hard bin a less precise evaluation of the same value could
 * change. */
int orc_mi_pmf(const float* F, const float* M, const float* u, i64 D, i64 H, i64 W, const i64* roi, int B,
               int hard, int pad, double* p_out, double edge_tol, i64* n_edge)
{
    const i64 N = D * H * W;
    i64 R[6];
    roi_or_full(roi, D, H, W, R);
    const double nroi = (double)((R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]));
    const int approx = hard == 2;
    double* acc = (double*)calloc((size_t)B * B, sizeof(double));
    i64 nedge = 0;
#pragma omp parallel reduction(+ : nedge)
    {
        double* pl = (double*)calloc((size_t)B * B, sizeof(double));
        double* kf = (double*)malloc(sizeof(double) * B);
        double* km = (double*)malloc(sizeof(double) * B);
        double* of = (double*)malloc(sizeof(double) * B);
        double* om = (double*)malloc(sizeof(double) * B);
#pragma omp for schedule(static)
        for (i64 z = R[0]; z < R[1]; ++z)
            for (i64 y = R[2]; y < R[3]; ++y)
                for (i64 x = R[4]; x < R[5]; ++x) {
                    const i64 k = AT(z, y, x);
                    double pt[3] = {(double)x, (double)y, (double)z};
                    if (u) { pt[0] += (double)u[k]; pt[1] += (double)u[N + k]; pt[2] += (double)u[2 * N + k]; }
                    const double mw = sample_point(M, D, H, W, pt, pad, NULL);
                    {
                        const double t = (mw < 0.0 ? 0.0 : (mw > 1.0 ? 1.0 : mw)) * (double)B;
                        const double e = floor(t + 0.5);
                        if (e > 0.0 && e < (double)B && fabs(t - e) <= edge_tol * (double)B) ++nedge;
                    }
                    if (approx) {
                        double vf = (double)F[k], vm = mw;
                        vf = vf < 0.0 ? 0.0 : (vf > 1.0 ? 1.0 : vf);
                        vm = vm < 0.0 ? 0.0 : (vm > 1.0 ? 1.0 : vm);
                        pl[hard_bin(vf, B) * B + hard_bin(vm, B)] += 1.0;
                        continue;
                    }
                    parzen_all((double)F[k], B, hard, kf, of);
                    parzen_all(mw, B, hard, km, om);
                    for (int m = 0; m < B; ++m) {
                        if (kf[m] == 0.0) continue;
                        for (int nn = 0; nn < B; ++nn) pl[m * B + nn] += kf[m] * km[nn];
                    }
                }
#pragma omp critical
        for (int q = 0; q < B * B; ++q) acc[q] += pl[q];
        free(pl); free(kf); free(km); free(of); free(om);
    }
    if (approx) {
        double* K = (double*)malloc(sizeof(double) * B * B);
        double* kc = (double*)malloc(sizeof(double) * B);
        double* oc = (double*)malloc(sizeof(double) * B);
        for (int j = 0; j < B; ++j) {
            parzen_all(((double)j + 0.5) / (double)B, B, 0, kc, oc);
            for (int m = 0; m < B; ++m) K[m * B + j] = kc[m];
        }
        for (int m = 0; m < B; ++m)
            for (int nn = 0; nn < B; ++nn) {
                double a = 0.0;
                for (int i = 0; i < B; ++i)
                    for (int j = 0; j < B; ++j) a += K[m * B + i] * K[nn * B + j] * acc[i * B + j];
                p_out[m * B + nn] = a / nroi;
            }
        free(K); free(kc); free(oc);
    } else {
        for (int q = 0; q < B * B; ++q) p_out[q] = acc[q] / nroi;
    }
    free(acc);
    if (n_edge) *n_edge = nedge;
    return 0;
}

/* dloss/du (loss = -MI) at the listed voxels pts [npts][3] (z, y, x), given
 * the joint PMF p of the same inputs (orc_mi_pmf): eq. gradientmi-threadn
 * with the full double sum of reading G7, times dMw/dp (O1):
 *   dloss/dMw_k = -(1/N_roi) sum_{m,n} kappa_m(F_k) omega_n(Mw_k)
 *                 (ln p[m][n] - ln pF[m] - ln pM[n] - 1)
 * (the last three terms sum to zero over n; ln p - ln pM is taken as 0 where
 * p = 0), zero outside the ROI.  hard = 2 uses the smooth kernel, as mi_core
 * does; hard = 1 gives zero. */
int orc_mi_grad_u_at(const float* F, const float* M, const float* u, i64 D, i64 H, i64 W, const i64* roi, int B,
                     int hard, int pad, const double* p, i64 npts, const i64* pts, double* out)
{
    const i64 N = D * H * W;
    i64 R[6];
    roi_or_full(roi, D, H, W, R);
    const double nroi = (double)((R[1] - R[0]) * (R[3] - R[2]) * (R[5] - R[4]));
    if (hard == 2) hard = 0;
    double* pF = (double*)calloc(B, sizeof(double));
    double* pM = (double*)calloc(B, sizeof(double));
    for (int m = 0; m < B; ++m)
        for (int nn = 0; nn < B; ++nn) { pF[m] += p[m * B + nn]; pM[nn] += p[m * B + nn]; }
    double* kf = (double*)malloc(sizeof(double) * B);
    double* km = (double*)malloc(sizeof(double) * B);
    double* of = (double*)malloc(sizeof(double) * B);
    double* om = (double*)malloc(sizeof(double) * B);
    for (i64 i = 0; i < npts; ++i) {
        const i64 z = pts[3 * i], y = pts[3 * i + 1], x = pts[3 * i + 2];
        out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = 0.0;
        if (!in_roi(R, z, y, x)) continue;
        const i64 k = AT(z, y, x);
        double pt[3] = {(double)x, (double)y, (double)z};
        if (u) { pt[0] += (double)u[k]; pt[1] += (double)u[N + k]; pt[2] += (double)u[2 * N + k]; }
        double dv[3];
        const double mw = sample_point(M, D, H, W, pt, pad, dv);
        parzen_all((double)F[k], B, hard, kf, of);
        parzen_all(mw, B, hard, km, om);
        double sdl = 0.0;
        for (int m = 0; m < B; ++m)
            for (int nn = 0; nn < B; ++nn) {
                const double wgt = kf[m] * om[nn];
                if (wgt == 0.0) continue;
                const double q = p[m * B + nn];
                const double t = q > 0.0 ? log(q) - log(pM[nn]) : 0.0;
                sdl += -wgt / nroi * (t - log(pF[m]) - 1.0);
            }
        out[3 * i] = sdl * dv[0];
        out[3 * i + 1] = sdl * dv[1];
        out[3 * i + 2] = sdl * dv[2];
    }
    free(pF); free(pM); free(kf); free(km); free(of); free(om);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O7. Composite implicit grid sampler (Sec. "Composite Implicit Grid        */
/* Sampler", the affine form of Alg. gridsampler): the sample point of the   */
/* target voxel X = (x, y, z) is p(X) = A X + t + S u(X), in voxel units,    */
/* A and S row-major 3x3 acting on (x, y, z) components; out(X) = M(p(X)).   */
/* Adjoint for an upstream gradient gout(X) = dL/dout(X):                    */
/*   dL/du(X) = S^T g(X),  dL/dA = sum_X g(X) X^T,  dL/dt = sum_X g(X),       */
/*   g(X) = gout(X) dM/dp(p(X)).                                             */
/* ------------------------------------------------------------------------ */
static void affine_point(const double* A, const double* t, const double* S, const float* u, i64 N, i64 k,
                         i64 x, i64 y, i64 z, double p[3])
{
    const double X[3] = {(double)x, (double)y, (double)z};
    double uu[3] = {0.0, 0.0, 0.0};
    if (u) { uu[0] = (double)u[k]; uu[1] = (double)u[N + k]; uu[2] = (double)u[2 * N + k]; }
    for (int i = 0; i < 3; ++i)
        p[i] = A[3 * i] * X[0] + A[3 * i + 1] * X[1] + A[3 * i + 2] * X[2] + t[i] +
               S[3 * i] * uu[0] + S[3 * i + 1] * uu[1] + S[3 * i + 2] * uu[2];
}

int orc_warp_affine(const float* M, const float* u, i64 D, i64 H, i64 W, const double* A, const double* t,
                    const double* S, int pad, double* out, double* dout)
{
    const i64 N = D * H * W;
#pragma omp parallel for schedule(static)
    for (i64 z = 0; z < D; ++z)
        for (i64 y = 0; y < H; ++y)
            for (i64 x = 0; x < W; ++x) {
                const i64 k = AT(z, y, x);
                double p[3], dv[3];
                affine_point(A, t, S, u, N, k, x, y, z, p);
                out[k] = sample_point(M, D, H, W, p, pad, dv);
                if (dout) { dout[k] = dv[0]; dout[N + k] = dv[1]; dout[2 * N + k] = dv[2]; }
            }
    return 0;
}

/* dL/du (nullable) and gAt[12] = (dL/dA row-major, dL/dt) from gout [N] and
 * the sampler derivative dM [3][N]. */
static void affine_adjoint(const double* S, const double* gout, const double* dM, i64 D, i64 H, i64 W,
                           double* grad_u, double* gAt)
{
    const i64 N = D * H * W;
    for (int q = 0; q < 12; ++q) gAt[q] = 0.0;
    for (i64 z = 0; z < D; ++z)
        for (i64 y = 0; y < H; ++y)
            for (i64 x = 0; x < W; ++x) {
                const i64 k = AT(z, y, x);
                const double X[3] = {(double)x, (double)y, (double)z};
                const double g[3] = {gout[k] * dM[k], gout[k] * dM[N + k], gout[k] * dM[2 * N + k]};
                for (int i = 0; i < 3; ++i) {
                    for (int j = 0; j < 3; ++j) gAt[3 * i + j] += g[i] * X[j];
                    gAt[9 + i] += g[i];
                }
                if (grad_u)
                    for (int j = 0; j < 3; ++j)
                        grad_u[j * N + k] = S[j] * g[0] + S[3 + j] * g[1] + S[6 + j] * g[2];
            }
}

int orc_warp_affine_bwd(const float* M, const float* u, i64 D, i64 H, i64 W, const double* A, const double* t,
                        const double* S, int pad, const double* gout, double* grad_u, double* gAt)
{
    const i64 N = D * H * W;
    double* out = (double*)malloc(sizeof(double) * N);
    double* dM = (double*)malloc(sizeof(double) * 3 * N);
    orc_warp_affine(M, u, D, H, W, A, t, S, pad, out, dM);
    affine_adjoint(S, gout, dM, D, H, W, grad_u, gAt);
    free(out); free(dM);
    return 0;
}

/* MI of (F, M(A X + t + S u)) with loss, PMF and the adjoint to u, A, t. */
int orc_mi_affine(const float* F, const float* M, const float* u, i64 D, i64 H, i64 W, const i64* roi,
                  const double* A, const double* t, const double* S, int B, int hard, int pad, double* loss,
                  double* p_out, double* grad_u, double* gAt)
{
    const i64 N = D * H * W;
    double* Mw = (double*)malloc(sizeof(double) * N);
    double* dM = (double*)malloc(sizeof(double) * 3 * N);
    double* s = (double*)malloc(sizeof(double) * N);
    orc_warp_affine(M, u, D, H, W, A, t, S, pad, Mw, dM);
    mi_core(F, Mw, D, H, W, roi, B, hard, loss, p_out, s);
    if (gAt) affine_adjoint(S, s, dM, D, H, W, grad_u, gAt);
    free(Mw); free(dM); free(s);
    return 0;
}

/* Parzen weights of one value (exported for the tests). */
int orc_parzen(double v, int B, int hard, double* kap, double* om)
{
    parzen_all(v, B, hard, kap, om);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O5. Adam (Kingma & Ba) with bias correction, the per-voxel optimiser with */
/* first and second moment states of the paper's registration loop.         */
/* ------------------------------------------------------------------------ */
int orc_adam(double* x, const double* g, double* m, double* v, i64 n, double lr, double b1, double b2,
             double eps, i64 step)
{
    const double bc1 = 1.0 - pow(b1, (double)step);
    const double bc2 = 1.0 - pow(b2, (double)step);
    for (i64 i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / bc1, vh = v[i] / bc2;
        x[i] -= lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Trilinear resize with corner alignment (multi-scale pyramid): dst voxel j */
/* samples src at j (n_src - 1)/(n_dst - 1) per axis; values are scaled by   */
/* value_scale (a displacement in voxels scales with the grid).              */
/* ------------------------------------------------------------------------ */
int orc_resample(const float* src, i64 sD, i64 sH, i64 sW, double* dst, i64 dD, i64 dH, i64 dW, int channels,
                 double value_scale)
{
    const i64 D = sD, H = sH, W = sW;
    const double fz = dD > 1 ? (double)(sD - 1) / (double)(dD - 1) : 0.0;
    const double fy = dH > 1 ? (double)(sH - 1) / (double)(dH - 1) : 0.0;
    const double fx = dW > 1 ? (double)(sW - 1) / (double)(dW - 1) : 0.0;
    for (int c = 0; c < channels; ++c) {
        const float* s = src + (i64)c * sD * sH * sW;
        double* d = dst + (i64)c * dD * dH * dW;
#pragma omp parallel for schedule(static)
        for (i64 z = 0; z < dD; ++z)
            for (i64 y = 0; y < dH; ++y)
                for (i64 x = 0; x < dW; ++x) {
                    double p[3] = {x * fx, y * fy, z * fz};
                    d[(z * dH + y) * dW + x] = value_scale * sample_point(s, D, H, W, p, 0, NULL);
                }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gaussian smoothing of a field (the sigma_grad / sigma_warp regulariser of */
/* the paper's registration runs): each output is the sum over the full      */
/* (2R+1)^3 neighbourhood of g(a) g(b) g(c) times the input at the offset,   */
/* indices clamped to the array (edge replication), with                     */
/* g(t) = exp(-t^2/(2 sigma^2)) / sum_{|s|<=R} exp(-s^2/(2 sigma^2)) and     */
/* R = ceil(3 sigma).  Direct triple sum, no separation.                     */
/* ------------------------------------------------------------------------ */
static i64 clampi(i64 v, i64 lo, i64 hi) { return v < lo ? lo : (v > hi ? hi : v); }

int orc_gaussian_smooth(const float* in, i64 D, i64 H, i64 W, int channels, double sigma, double* out)
{
    if (!(sigma > 0.0)) return 1;
    const int R = (int)ceil(3.0 * sigma);
    double* g = (double*)malloc(sizeof(double) * (2 * R + 1));
    double tot = 0.0;
    for (int t = -R; t <= R; ++t) tot += (g[t + R] = exp(-(double)(t * t) / (2.0 * sigma * sigma)));
    for (int t = 0; t <= 2 * R; ++t) g[t] /= tot;
    for (int c = 0; c < channels; ++c) {
        const float* s = in + (i64)c * D * H * W;
        double* o = out + (i64)c * D * H * W;
#pragma omp parallel for schedule(static)
        for (i64 z = 0; z < D; ++z)
            for (i64 y = 0; y < H; ++y)
                for (i64 x = 0; x < W; ++x) {
                    double acc = 0.0;
                    for (int a = -R; a <= R; ++a)
                        for (int b = -R; b <= R; ++b)
                            for (int e = -R; e <= R; ++e)
                                acc += g[a + R] * g[b + R] * g[e + R] *
                                       (double)s[AT(clampi(z + a, 0, D - 1), clampi(y + b, 0, H - 1),
                                                    clampi(x + e, 0, W - 1))];
                    o[AT(z, y, x)] = acc;
                }
    }
    free(g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O6. 3x3x3 convolution of the warm-start network (zero padding 1, stride   */
/* s), in double on operands the caller has already rounded to bf16.  The    */
/* input X is the channel concatenation of part a (nearest x2 upsampled when */
/* ups = 1) and part b; layouts are channels-last [N][D][H][W][C]; the       */
/* weight is [Cout][27][Cin] with tap t = (dz*3 + dy)*3 + dx.                */
/* ------------------------------------------------------------------------ */
typedef struct {
    i64 N, Di, Hi, Wi, Do, Ho, Wo, Ca, Cb, Cout, s, ups;
} cgeo;

static cgeo mkgeo(i64 N, i64 Di, i64 Hi, i64 Wi, i64 Ca, i64 Cb, i64 Cout, i64 s, i64 ups)
{
    cgeo g = {N, Di, Hi, Wi, (Di - 1) / s + 1, (Hi - 1) / s + 1, (Wi - 1) / s + 1, Ca, Cb, Cout, s, ups};
    return g;
}

/* X[n][z][y][x][c] by its definition */
static double xin(const cgeo* g, const double* xa, const double* xb, i64 n, i64 z, i64 y, i64 x, i64 c)
{
    if (c < g->Ca) {
        if (g->ups) {
            i64 Da = g->Di / 2, Ha = g->Hi / 2, Wa = g->Wi / 2;
            return xa[((((n * Da) + z / 2) * Ha + y / 2) * Wa + x / 2) * g->Ca + c];
        }
        return xa[((((n * g->Di) + z) * g->Hi + y) * g->Wi + x) * g->Ca + c];
    }
    return xb[((((n * g->Di) + z) * g->Hi + y) * g->Wi + x) * g->Cb + (c - g->Ca)];
}

int orc_conv3d_fwd(const double* xa, const double* xb, const double* w, const double* bias, i64 N, i64 Di, i64 Hi,
                   i64 Wi, i64 Ca, i64 Cb, i64 Cout, i64 s, i64 ups, int act, double slope, double* y)
{
    cgeo g = mkgeo(N, Di, Hi, Wi, Ca, Cb, Cout, s, ups);
    const i64 Cin = Ca + Cb;
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 n = 0; n < N; ++n)
        for (i64 zo = 0; zo < g.Do; ++zo)
            for (i64 yo = 0; yo < g.Ho; ++yo)
                for (i64 xo = 0; xo < g.Wo; ++xo)
                    for (i64 co = 0; co < Cout; ++co) {
                        double acc = bias ? bias[co] : 0.0;
                        for (i64 t = 0; t < 27; ++t) {
                            i64 zi = zo * s + t / 9 - 1, yi = yo * s + (t / 3) % 3 - 1, xi = xo * s + t % 3 - 1;
                            if (zi < 0 || zi >= Di || yi < 0 || yi >= Hi || xi < 0 || xi >= Wi) continue;
                            for (i64 ci = 0; ci < Cin; ++ci)
                                acc += xin(&g, xa, xb, n, zi, yi, xi, ci) * w[(co * 27 + t) * Cin + ci];
                        }
                        if (act && acc <= 0.0) acc *= slope;
                        y[((((n * g.Do) + zo) * g.Ho + yo) * g.Wo + xo) * Cout + co] = acc;
                    }
    return 0;
}

/* Adjoint of the convolution with respect to X (scatter form): every output
 * voxel o and tap t send P[o][co] w[co][t][ci] to input voxel o*s + t - 1.
 * dx is over the concatenated fine-resolution input, [N][Di][Hi][Wi][Ca+Cb]. */
int orc_conv3d_bwd_data(const double* P, const double* w, i64 N, i64 Di, i64 Hi, i64 Wi, i64 Ca, i64 Cb, i64 Cout,
                        i64 s, double* dx)
{
    cgeo g = mkgeo(N, Di, Hi, Wi, Ca, Cb, Cout, s, 0);
    const i64 Cin = Ca + Cb;
    memset(dx, 0, sizeof(double) * (size_t)(N * Di * Hi * Wi * Cin));
    for (i64 n = 0; n < N; ++n)
        for (i64 zo = 0; zo < g.Do; ++zo)
            for (i64 yo = 0; yo < g.Ho; ++yo)
                for (i64 xo = 0; xo < g.Wo; ++xo)
                    for (i64 t = 0; t < 27; ++t) {
                        i64 zi = zo * s + t / 9 - 1, yi = yo * s + (t / 3) % 3 - 1, xi = xo * s + t % 3 - 1;
                        if (zi < 0 || zi >= Di || yi < 0 || yi >= Hi || xi < 0 || xi >= Wi) continue;
                        double* d = dx + ((((n * Di) + zi) * Hi + yi) * Wi + xi) * Cin;
                        const double* p = P + ((((n * g.Do) + zo) * g.Ho + yo) * g.Wo + xo) * Cout;
                        for (i64 co = 0; co < Cout; ++co)
                            for (i64 ci = 0; ci < Cin; ++ci) d[ci] += p[co] * w[(co * 27 + t) * Cin + ci];
                    }
    return 0;
}

/* dW[co][t][ci] = sum_o P[o][co] X[o*s + t - 1][ci];  db[co] = sum_o P[o][co] */
int orc_conv3d_bwd_weight(const double* xa, const double* xb, const double* P, i64 N, i64 Di, i64 Hi, i64 Wi, i64 Ca,
                          i64 Cb, i64 Cout, i64 s, i64 ups, double* dw, double* db)
{
    cgeo g = mkgeo(N, Di, Hi, Wi, Ca, Cb, Cout, s, ups);
    const i64 Cin = Ca + Cb;
#pragma omp parallel for schedule(static)
    for (i64 co = 0; co < Cout; ++co) {
        for (i64 q = 0; q < 27 * Cin; ++q) dw[co * 27 * Cin + q] = 0.0;
        double b = 0.0;
        for (i64 n = 0; n < N; ++n)
            for (i64 zo = 0; zo < g.Do; ++zo)
                for (i64 yo = 0; yo < g.Ho; ++yo)
                    for (i64 xo = 0; xo < g.Wo; ++xo) {
                        double p = P[((((n * g.Do) + zo) * g.Ho + yo) * g.Wo + xo) * Cout + co];
                        b += p;
                        for (i64 t = 0; t < 27; ++t) {
                            i64 zi = zo * s + t / 9 - 1, yi = yo * s + (t / 3) % 3 - 1, xi = xo * s + t % 3 - 1;
                            if (zi < 0 || zi >= Di || yi < 0 || yi >= Hi || xi < 0 || xi >= Wi) continue;
                            for (i64 ci = 0; ci < Cin; ++ci)
                                dw[(co * 27 + t) * Cin + ci] += p * xin(&g, xa, xb, n, zi, yi, xi, ci);
                        }
                    }
        if (db) db[co] = b;
    }
    return 0;
}

/* Host threads of the OpenMP loops (timing of the oracle at a given width). */
int orc_set_threads(int n)
{
    if (n < 1) return -1;
    omp_set_num_threads(n);
    return 0;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
