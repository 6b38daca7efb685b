/*
 * ffdp.h — C ABI of the fused warp + dissimilarity library for MI355X (gfx950).
 *
 * The library computes the data-parallel hot path of deformable image
 * registration in the paper's formulation (Sec. "Composite Implicit Grid
 * Sampler", App. "Fused LNCC", App. "Implicit MI"): the moving volume M is
 * sampled trilinearly at the implicit identity grid plus a displacement u,
 * never materialising a grid, and compared with the fixed volume F by local
 * normalised cross-correlation (LNCC) or Parzen-window mutual information
 * (MI); the hand-written adjoint returns dloss/du and a per-voxel Adam step
 * updates u.
 *
 * Common conventions (every entry point):
 *  - Volumes are float32, C-order [D][H][W] (z, y, x), contiguous.
 *    Displacements and their gradients are [3][D][H][W]; channel 0 adds to
 *    x (the W axis), channel 1 to y (H), channel 2 to z (D), in voxel units
 *    (Alg. gridsampler: X = (x, y, z), displacement u[:, z, y, x]).
 *  - All data pointers are DEVICE pointers, 4-byte aligned, owned by the
 *    caller.  The library never allocates device memory: scratch comes from
 *    a caller workspace whose size the *_workspace_bytes queries return
 *    (it grows with the number of thread blocks, never with the voxel count).
 *  - D*H*W must be below 2^31.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Arguments are validated on the host before anything is
 *    launched; on error nothing is launched and outputs are untouched.
 *  - Return value: FFDP_OK or one of the FFDP_ERR_* codes below.  The text
 *    of the last error on the calling thread is in ffdp_last_error().
 *  - Calls on different streams with disjoint outputs and workspaces may run
 *    concurrently; the library keeps no mutable global state, except for
 *    the one entry point for callers that cannot allocate
 *    (ffdp_warp_lncc_bwd_noalloc), whose scratch array is shared per GPU.
 *  - Reductions are two-stage and in a fixed order (LNCC) or in exact
 *    integer arithmetic (MI histogram), so results are bitwise reproducible.
 */
#ifndef FFDP_H
#define FFDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFDP_OK 0
#define FFDP_ERR_NULL 1      /* a required pointer is NULL */
#define FFDP_ERR_SHAPE 2     /* bad dimensions or ROI */
#define FFDP_ERR_PARAM 3     /* bad window, eps, bins, pad mode, lr, step ... */
#define FFDP_ERR_ALIGN 4     /* a pointer is not 4-byte aligned */
#define FFDP_ERR_WORKSPACE 5 /* workspace NULL or smaller than the query */
#define FFDP_ERR_HIP 6       /* the HIP runtime refused a launch */
#define FFDP_ERR_NONFINITE 7 /* checked mode: a NaN or infinite input, or a non-finite loss */

#define FFDP_PAD_BORDER 0 /* samples clamp to the array (default) */
#define FFDP_PAD_ZEROS 1  /* lattice points outside the array read as 0 */

/* Array geometry and the loss region (ROI), all in (z, y, x) order.  The ROI
 * is the half-open box [roi_lo, roi_hi); it must be non-empty and inside the
 * array.  Window sums read real array values around the ROI (the halo) and
 * zeros outside the array. */
typedef struct ffdp_grid {
    int64_t D, H, W;
    int64_t roi_lo[3];
    int64_t roi_hi[3];
} ffdp_grid;

/* Checked mode (check_finite = 1 in the parameters of ffdp_warp_lncc_fwd,
 * ffdp_warp_lncc_bwd, ffdp_warp_mi_fwd and ffdp_warp_mi_bwd): before the
 * computation a pass over F, M, u (when given) and grad_scale (when given)
 * flags NaN and infinite values; after it the call WAITS for the stream
 * (the only calls that do) and returns FFDP_ERR_NONFINITE if an input was
 * flagged or the loss it wrote is not finite (finite inputs can still give a
 * NaN loss, e.g. eps = 0 with a constant window).  The outputs are written
 * either way.  The flag lives in the caller's workspace.  0: no checks, no
 * wait (the default). */

/* LNCC settings (App. "Definition of LNCC loss", Alg. fusedlncc):
 *  window       odd box edge w in [3, 15]; the filter is the uniform w^3 box
 *               with weights 1/w^3, zero padding at the array border.
 *               w <= 9 runs one fused kernel per call; w = 11, 13, 15 run
 *               separable passes through an FP64 workspace of 64 bytes per
 *               voxel (the fused kernel's register rings do not fit there).
 *  eps          the stabiliser in n_i = A_i^2 / (B_i C_i + eps); >= 0.
 *  ants_approx  1: skip the window sum of the adjoint (App. "ANTs gradient
 *               approximation"); 0: exact gradient.
 *  pad_mode     FFDP_PAD_BORDER or FFDP_PAD_ZEROS for the sampler.
 *  check_finite 0 or 1 (checked mode, above). */
typedef struct ffdp_lncc_params {
    int32_t window;
    float eps;
    int32_t ants_approx;
    int32_t pad_mode;
    int32_t check_finite;
} ffdp_lncc_params;

/* MI settings (eq. mi, App. "Vanilla MI implementation"):
 *  bins      B in [8, 256]; bin centres (m + 1/2)/B on [0, 1]; intensities
 *            are clamped to [0, 1].  The kernel is the cubic B-spline of one
 *            bin width; support beyond the first/last bin folds onto it.
 *  hard_bins 0: the Parzen estimate above.
 *            1: box kernel (one bin per voxel, zero gradient) — test mode.
 *            2: the approximate estimator (App. "Implicit MI implementation",
 *               approximate histogram estimator): each voxel counts once in
 *               bin min(floor(v B), B-1) (fp32); the count histogram over the
 *               ROI is normalised and convolved with the kernel at bin-centre
 *               offsets (taps 1/6, 2/3, 1/6, folded like the kernel).  The
 *               backward pass is the hard_bins = 0 one evaluated with this p.
 *  pad_mode  as for LNCC.
 *  check_finite 0 or 1 (checked mode, above; ffdp_warp_mi_fwd and
 *            ffdp_warp_mi_bwd only, 0 for the composite-sampler calls). */
typedef struct ffdp_mi_params {
    int32_t bins;
    int32_t hard_bins;
    int32_t pad_mode;
    int32_t check_finite;
} ffdp_mi_params;

/* Library version (major*10000 + minor*100 + patch). */
int ffdp_version(void);
/* Static text for a status code. */
const char* ffdp_status_string(int status);
/* Text of the last error on this thread ("" if none). */
const char* ffdp_last_error(void);

/* Workspace bytes for the LNCC / MI calls on this geometry (0 never occurs):
 * LNCC w <= 9: 8 per thread block of the launch plus 16 (checked-mode flag);
 * LNCC w >= 11: 64 per voxel (FP64 window sums and adjoint fields) plus 8
 * per block of its column passes plus 16; MI 8 * (B^2 + 2).  With p NULL or
 * invalid: enough for any valid p (the wide-window size for LNCC). */
size_t ffdp_lncc_workspace_bytes(const ffdp_grid* g, const ffdp_lncc_params* p);
size_t ffdp_mi_workspace_bytes(const ffdp_grid* g, const ffdp_mi_params* p);
/* Number of floats in the caller-owned MI state: 2*B*B + 2*B + 16. */
size_t ffdp_mi_state_floats(int32_t bins);

/* Composite implicit grid sampler, identity + displacement case
 * (Sec. "Composite Implicit Grid Sampler", Alg. gridsampler Forward):
 *   out(x) = M(x + u(x)) by trilinear interpolation (eq. interp).
 * M [D][H][W]; u [3][D][H][W] or NULL (zero displacement); out [D][H][W].
 * The ROI fields of g are ignored. */
int ffdp_warp(const float* M, const float* u, const ffdp_grid* g, int32_t pad_mode, float* out, void* stream);

/* Trilinear resize with corner alignment, the multi-scale pyramid step of the
 * paper's registration loop: dst voxel j samples src at j*(n_src-1)/(n_dst-1)
 * per axis; every value is multiplied by value_scale (2.0 when a displacement
 * in voxels moves to a grid twice as fine).  src [channels][sD][sH][sW],
 * dst [channels][dD][dH][dW]; src and dst must not overlap. */
int ffdp_resample(const float* src, int64_t sD, int64_t sH, int64_t sW, float* dst, int64_t dD, int64_t dH,
                  int64_t dW, int32_t channels, float value_scale, void* stream);

/* Fused warp + LNCC forward (Alg. fusedlncc Forward with the sampler fused in):
 *   loss = 1 - (1/N_roi) sum_{i in ROI} A_i^2/(B_i C_i + eps)
 * with A, B, C the windowed covariance/variances of F and M(x + u).
 * *loss (one device float) receives the value; ws/ws_bytes as queried. */
int ffdp_warp_lncc_fwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                       const ffdp_lncc_params* p, float* loss, void* ws, size_t ws_bytes, void* stream);

/* Fused warp + LNCC forward and adjoint in one pass (Alg. fusedlncc Backward,
 * eq. finalccgradM, Alg. gridsampler Backward for the displacement):
 *   grad_u = grad_scale * dloss/du, OVERWRITTEN over the whole array (zero
 *   where no window of the ROI reaches).
 * grad_scale: device float or NULL (= 1).  loss: device float or NULL; when
 * given it receives the same value as ffdp_warp_lncc_fwd. */
int ffdp_warp_lncc_bwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                       const ffdp_lncc_params* p, const float* grad_scale, float* grad_u, float* loss, void* ws,
                       size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): ffdp_warp_lncc_bwd with its block partials in a library-owned
 * device array of FFDP_NOALLOC_MAX_BLOCKS doubles (512 KB, one per GPU, held
 * until the process ends) instead of a caller workspace.  Same arguments and
 * results otherwise (bitwise the same outputs; checked mode included).  Calls
 * whose workspace (ffdp_lncc_workspace_bytes) exceeds the array are rejected
 * with FFDP_ERR_WORKSPACE before anything runs: grids needing more than
 * FFDP_NOALLOC_MAX_BLOCKS block partials, and wide windows (w >= 11) beyond
 * about 8,000 voxels.  All calls on one
 * GPU share its array: calls that overlap in time on one GPU (different
 * streams or threads) race and must be serialised by the caller.  The array
 * belongs to the device that runs `stream`. */
#define FFDP_NOALLOC_MAX_BLOCKS 65536
int ffdp_warp_lncc_bwd_noalloc(const float* F, const float* M, const float* u, const ffdp_grid* g,
                               const ffdp_lncc_params* p, const float* grad_scale, float* grad_u, float* loss,
                               void* stream);

/* Fused warp + Parzen MI forward (eq. mi; App. "Implicit MI implementation",
 * Forward Pass): the joint histogram of (F, M(x+u)) over the ROI, then
 *   loss = -MI = -sum p log(p / (p_F p_M)).
 * mi_state (ffdp_mi_state_floats(bins) device floats, caller-owned) receives
 *   [0, B*B)            T[m][n] = log p[m][n] - log p_M[n] (0 where p = 0)
 *   [B*B, 2*B*B)        p[m][n] (m: F bin, n: warped-M bin)
 *   [2B*B, 2B*B+B)      p_F;   [2B*B+B, 2B*B+2B) p_M
 *   [2B*B+2B] loss, [+1] MI, [+2] bins, rest reserved.
 * loss: device float (may point into mi_state). */
int ffdp_warp_mi_fwd(const float* F, const float* M, const float* u, const ffdp_grid* g, const ffdp_mi_params* p,
                     float* loss, float* mi_state, void* ws, size_t ws_bytes, void* stream);

/* MI adjoint (App. "Implicit MI implementation", Backward Pass, with the
 * sampler adjoint): grad_u = grad_scale * dloss/du, OVERWRITTEN over the whole
 * array (zero outside the ROI).  mi_state must come from ffdp_warp_mi_fwd on
 * the same F, M, u and parameters (a stale state gives a wrong gradient). */
int ffdp_warp_mi_bwd(const float* F, const float* M, const float* u, const ffdp_grid* g, const ffdp_mi_params* p,
                     const float* mi_state, const float* grad_scale, float* grad_u, void* ws, size_t ws_bytes,
                     void* stream);

/* Affine part of the composite implicit grid sampler (Sec. "Composite
 * Implicit Grid Sampler"): the sample point of target voxel X = (x, y, z) is
 *   p(X) = A X + t + S u(X)       (voxel units; A, S row-major 3x3 acting on
 *                                  (x, y, z) and (u_x, u_y, u_z) components)
 * A = S = I, t = 0 is the identity sampler of the other entry points.  All
 * values must be finite. */
typedef struct ffdp_affine {
    float A[9];
    float t[3];
    float S[9];
} ffdp_affine;

/* Bytes of the caller workspace for the composite-sampler adjoints
 * (per-block partial sums of dL/dA and dL/dt; grows with the block count). */
size_t ffdp_affine_workspace_bytes(const ffdp_grid* g);

/* Composite sampler forward: out(X) = M(p(X)) by trilinear interpolation
 * (eq. interp), never materialising p.  M, out [D][H][W]; u [3][D][H][W] or
 * NULL (affine only); the ROI fields of g are ignored. */
int ffdp_warp_affine(const float* M, const float* u, const ffdp_grid* g, const ffdp_affine* aff, int32_t pad_mode,
                     float* out, void* stream);

/* Composite sampler adjoint for an upstream gradient gout = dL/dout
 * [D][H][W] (the affine form of Alg. gridsampler Backward):
 *   grad_u(X) = S^T g(X)  with g(X) = gout(X) dM/dp(p(X))   (skipped if NULL)
 *   grad_At[0..8] = sum_X g(X) X^T (dL/dA, row-major), grad_At[9..11] = sum_X g(X)
 * grad_At: 12 device doubles, overwritten, summed in a fixed order
 * (bitwise reproducible).  ws: ffdp_affine_workspace_bytes(g), 8-byte aligned. */
int ffdp_warp_affine_bwd(const float* M, const float* u, const ffdp_grid* g, const ffdp_affine* aff,
                         int32_t pad_mode, const float* gout, float* grad_u, double* grad_At, void* ws,
                         size_t ws_bytes, void* stream);

/* Warp + MI forward through the composite sampler (the affine MI stage of
 * the paper's pipeline): as ffdp_warp_mi_fwd with Mw(X) = M(p(X)).
 * ws: ffdp_mi_workspace_bytes. */
int ffdp_warp_mi_affine_fwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                            const ffdp_affine* aff, const ffdp_mi_params* p, float* loss, float* mi_state, void* ws,
                            size_t ws_bytes, void* stream);

/* MI adjoint through the composite sampler: grad_u (nullable) as
 * ffdp_warp_mi_bwd times S^T, grad_At (12 device doubles) = dL/dA, dL/dt
 * as in ffdp_warp_affine_bwd with gout = dL/dMw.  mi_state from
 * ffdp_warp_mi_affine_fwd with the same arguments.
 * ws: ffdp_affine_workspace_bytes(g). */
int ffdp_warp_mi_affine_bwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                            const ffdp_affine* aff, const ffdp_mi_params* p, const float* mi_state,
                            const float* grad_scale, float* grad_u, double* grad_At, void* ws, size_t ws_bytes,
                            void* stream);

/* Per-element Adam with bias correction, the optimiser with first and second
 * moment states that the paper shards with the displacement (Sec. "Grid
 * Parallel"), in place on x, m, v over n elements:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   x -= lr (m/(1-b1^step)) / (sqrt(v/(1-b2^step)) + eps)
 * step >= 1; 0 <= b1, b2 < 1; eps > 0.  Also used for network weights. */
int ffdp_adam_step(float* x, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                   float eps, int64_t step, void* stream);

/* Gaussian smoothing of a multi-channel field, the regulariser applied to the
 * displacement gradient (sigma_grad = 1) before the optimiser step and to the
 * displacement (sigma_warp = 0.5) after it in the paper's registration runs
 * (Sec. "Grid Parallel", App. experiment settings):
 *   out[c] = g * g * g (separable) applied to in[c], per channel, with
 *   g(t) = exp(-t^2 / (2 sigma^2)) / sum_{|s| <= R} exp(-s^2 / (2 sigma^2)),
 *   |t| <= R = ceil(3 sigma), and the array edge value replicated outside.
 * in, out [channels][D][H][W]; they must not overlap.  0 < sigma <= 2. */
int ffdp_gaussian_smooth(const float* in, float* out, int64_t D, int64_t H, int64_t W, int32_t channels, float sigma,
                         void* stream);

/* One optimiser step of the registration loop with the gradient smoothed
 * first (Sec. "Grid Parallel"; sigma_grad = 1 in the experiments): exactly
 * ffdp_gaussian_smooth(g -> s, sigma) followed by ffdp_adam_step(x, s, m, v)
 * on the same [channels][D][H][W] arrays, bitwise, without writing s.
 * x, m, v are updated in place; g is read only and must not overlap x, m or
 * v (nor may x, m, v overlap each other).  Parameter rules as for those two
 * calls. */
int ffdp_smooth_adam_step(float* x, const float* g, float* m, float* v, int64_t D, int64_t H, int64_t W,
                          int32_t channels, float sigma, float lr, float beta1, float beta2, float eps, int64_t step,
                          void* stream);

/* ------------------------------------------------------------------------
 * Warm-start network (3D U-Net) kernels.  The paper trains a learned
 * registration network with its fused losses (App. "Accelerating TransMorph
 * training") but specifies no architecture; this network, which predicts an
 * initial displacement for the optimisation, is this library's own.  The
 * operations are the textbook 3x3x3 convolution, its two adjoints (to the
 * input and to the weights) and LeakyReLU.  BF16 operands on MFMA with FP32
 * accumulation.  Activations are channels-last bf16 [N][D][H][W][C]
 * (uint16_t holding bfloat16 bits).  All convolutions are 3x3x3 with zero
 * padding 1 and stride 1 or 2; output size Do = (Di - 1)/stride + 1 per axis.
 * The convolution input may be the channel concatenation of part a
 * (channels [0, Ca)) and part b (channels [Ca, Ca + Cb)); with ups = 1 part a
 * is stored at half resolution (Di/2, Hi/2, Wi/2) and upsampled by nearest
 * x2 on the fly.  Channel counts Ca, Cb, Cout are multiples of 4;
 * Ca + Cb <= 192, Cout <= 128.  Pointers to bf16 data are 8-byte aligned,
 * fp32 gradient tensors 16-byte aligned.
 * ------------------------------------------------------------------------ */
typedef struct ffdp_conv_geom {
    int32_t N;
    int32_t Di, Hi, Wi; /* convolution input size (after upsampling) */
    int32_t Ca, Cb;     /* channels of part a and part b (0: no part b) */
    int32_t Cout;
    int32_t stride;     /* 1 or 2 */
    int32_t ups;        /* 1: part a is upsampled x2 (Di, Hi, Wi even) */
    /* N * Di * Hi * Wi below 2^31 (voxel indices are 32-bit) */
} ffdp_conv_geom;

/* Forward: y[o][co] = act(bias[co] + sum_{t, ci} X[o*stride + t - 1][ci] * w[co][t][ci]).
 * w bf16 [Cout][27][Cin] (t = (dz*3 + dy)*3 + dx); bias fp32 [Cout] or NULL;
 * act 1 = LeakyReLU with `slope`, 0 = identity.  y_bf16 and/or y_f32
 * [N][Do][Ho][Wo][Cout] (at least one non-NULL). */
int ffdp_conv3d_fwd(const uint16_t* xa, const uint16_t* xb, const uint16_t* w, const float* bias,
                    const ffdp_conv_geom* g, int32_t act, float slope, uint16_t* y_bf16, float* y_f32, void* stream);

/* Backward to the input: dx[i][ci] (+)= sum_{t, co} P[(i + 1 - t)/stride][co] * w[co][t][ci]
 * (terms with a non-integer or out-of-range output index are absent), where
 * P = bf16(dy * act'(y)) with act'(y) = 1 where y > 0 else slope (y = the
 * layer's bf16 output, or NULL for no activation).  wt is the weight in
 * [Cin][27][Cout] order (ffdp_conv3d_weight_prep).  dy fp32
 * [N][Do][Ho][Wo][Cout]; dx fp32 [N][Di][Hi][Wi][Ca + Cb] over the
 * concatenated fine-resolution input (ffdp_concat_grad_split separates it);
 * accumulate 1 adds to dx. */
int ffdp_conv3d_bwd_data(const float* dy, const uint16_t* y, float slope, const uint16_t* wt,
                         const ffdp_conv_geom* g, float* dx, int32_t accumulate, void* stream);

/* P = bf16(dy * act'(y)) elementwise over n elements (y NULL: act' = 1),
 * rounded to nearest even as the backward kernels round their operands; dy
 * fp32, y and p bf16, all in the same layout (e.g. [N][Do][Ho][Wo][Cout]).
 * Lets a layer's backward form P once for ffdp_conv3d_bwd_data_bf16. */
int ffdp_conv3d_act_grad(const float* dy, const uint16_t* y, float slope, int64_t n, uint16_t* p, void* stream);

/* ffdp_conv3d_bwd_data with P given directly: p bf16 [N][Do][Ho][Wo][Cout]
 * (16-byte aligned), e.g. from ffdp_conv3d_act_grad.  Bitwise the same dx
 * as ffdp_conv3d_bwd_data(dy, y, slope, ...) for p = act_grad(dy, y, slope);
 * one 16-byte operand load per lane and K step instead of three plus the
 * conversion. */
int ffdp_conv3d_bwd_data_bf16(const uint16_t* p, const uint16_t* wt, const ffdp_conv_geom* g, float* dx,
                              int32_t accumulate, void* stream);

/* Backward to the weights: dw[co][t][ci] = sum_o P[o][co] X[o*stride + t - 1][ci]
 * and db[co] = sum_o P[o][co] (db may be NULL), fp32, overwritten; the sums
 * over output voxels run in chunks whose partials (caller workspace) are
 * added in a fixed order.  For the stride-2 layers and those with more than
 * 64 output channels the workspace also holds P as bf16 in [Cout][voxel]
 * order (2 bytes per output voxel and channel). */
/* ffdp_conv3d_bwd_weight with P given directly: p bf16 [N][Do][Ho][Wo][Cout]
 * (8-byte aligned), e.g. from ffdp_conv3d_act_grad; the same workspace.  The
 * same dw and db, bit for bit, as ffdp_conv3d_bwd_weight(dy, y, slope, ...)
 * for p = act_grad(dy, y, slope). */
int ffdp_conv3d_bwd_weight_bf16(const uint16_t* xa, const uint16_t* xb, const uint16_t* p, const ffdp_conv_geom* g,
                                float* dw, float* db, void* ws, size_t ws_bytes, void* stream);

size_t ffdp_conv3d_bwd_weight_workspace_bytes(const ffdp_conv_geom* g);
int ffdp_conv3d_bwd_weight(const uint16_t* xa, const uint16_t* xb, const float* dy, const uint16_t* y, float slope,
                           const ffdp_conv_geom* g, float* dw, float* db, void* ws, size_t ws_bytes, void* stream);

/* fp32 master weights [Cout][27][Cin] -> bf16 copy (w_bf16, nullable) and
 * bf16 transpose [Cin][27][Cout] (wt_bf16, nullable), round to nearest even. */
int ffdp_conv3d_weight_prep(const float* w, int32_t Cout, int32_t Cin, uint16_t* w_bf16, uint16_t* wt_bf16,
                            void* stream);

/* Network input: (F, M) fp32 volumes of nvox voxels each (batch included)
 * -> bf16 [nvox][4] = (F, M, 0, 0). */
int ffdp_unet_pack_pair(const float* F, const float* M, int64_t nvox, uint16_t* x, void* stream);

/* Split dx of a concatenated input (layout of ffdp_conv3d_bwd_data) into the
 * skip part dxb [N][Di][Hi][Wi][Cb] and part a, summed over each 2x2x2 block
 * when ups = 1 (the adjoint of nearest upsampling) into dxa
 * [N][Di/2][Hi/2][Wi/2][Ca]; acc_a / acc_b = 1 add instead of overwrite.
 * All three pointers 16-byte aligned (FFDP_ERR_ALIGN otherwise). */
int ffdp_concat_grad_split(const float* dxcat, const ffdp_conv_geom* g, float* dxa, float* dxb, int32_t acc_a,
                           int32_t acc_b, void* stream);

/* Mean squared error between the first 3 channels of pred [N][nvox][Cp] and
 * target [N][3][nvox]: *loss = mean over N*3*nvox; dpred (nullable) receives
 * the gradient (channels >= 3 zero).  ws: ffdp_mse_workspace_bytes(). */
size_t ffdp_mse_workspace_bytes(void);
int ffdp_mse_disp(const float* pred, int32_t Cp, const float* target, int64_t nvox, int32_t N, float* dpred,
                  float* loss, void* ws, size_t ws_bytes, void* stream);

/* pred [N][nvox][Cp] -> displacement [N][3][nvox] (channels 0..2). */
int ffdp_unpack_disp(const float* pred, int32_t Cp, int64_t nvox, int32_t N, float* u, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FFDP_H */
