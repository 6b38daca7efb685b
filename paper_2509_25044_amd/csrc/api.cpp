// C-ABI entry points: host-side validation, workspace layout, dispatch.
// Nothing here allocates device memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/ffdp.h"
#include "adam.hpp"
#include "internal.hpp"
#include "wide.hpp"
#include "conv_p.hpp"

using namespace ffdp;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return FFDP_OK;
    return fail(FFDP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool misaligned(const void* p) { return (((uintptr_t)p) & 3u) != 0; }

constexpr int64_t MAX_VOXELS = 2147483647LL;  // 32-bit element offsets per channel

int check_dims(int64_t D, int64_t H, int64_t W)
{
    if (D < 1 || H < 1 || W < 1) return fail(FFDP_ERR_SHAPE, "dimensions must be >= 1 (got %lld x %lld x %lld)",
                                             (long long)D, (long long)H, (long long)W);
    if (H > 65535) return fail(FFDP_ERR_SHAPE, "H must be <= 65535");
    if (D > MAX_VOXELS / H || D * H > MAX_VOXELS / W)
        return fail(FFDP_ERR_SHAPE, "D*H*W must be below 2^31");
    return FFDP_OK;
}

int check_grid(const ffdp_grid* g)
{
    if (!g) return fail(FFDP_ERR_NULL, "grid is NULL");
    int s = check_dims(g->D, g->H, g->W);
    if (s) return s;
    const int64_t n[3] = {g->D, g->H, g->W};
    for (int k = 0; k < 3; ++k)
        if (g->roi_lo[k] < 0 || g->roi_hi[k] > n[k] || g->roi_lo[k] >= g->roi_hi[k])
            return fail(FFDP_ERR_SHAPE, "ROI axis %d [%lld, %lld) is empty or outside [0, %lld)", k,
                        (long long)g->roi_lo[k], (long long)g->roi_hi[k], (long long)n[k]);
    return FFDP_OK;
}

int check_lncc(const ffdp_lncc_params* p)
{
    if (!p) return fail(FFDP_ERR_NULL, "lncc params are NULL");
    if (p->window < 3 || p->window > LNCC_MAX_WINDOW || !(p->window & 1))
        return fail(FFDP_ERR_PARAM, "window must be odd in [3, %d] (got %d)", LNCC_MAX_WINDOW, p->window);
    if (!(p->eps >= 0.0f) || isinf(p->eps)) return fail(FFDP_ERR_PARAM, "eps must be finite and >= 0");
    if (p->ants_approx != 0 && p->ants_approx != 1) return fail(FFDP_ERR_PARAM, "ants_approx must be 0 or 1");
    if (p->pad_mode != FFDP_PAD_BORDER && p->pad_mode != FFDP_PAD_ZEROS)
        return fail(FFDP_ERR_PARAM, "pad_mode must be 0 (border) or 1 (zeros)");
    if (p->check_finite != 0 && p->check_finite != 1) return fail(FFDP_ERR_PARAM, "check_finite must be 0 or 1");
    return FFDP_OK;
}

int check_mi(const ffdp_mi_params* p)
{
    if (!p) return fail(FFDP_ERR_NULL, "mi params are NULL");
    if (p->bins < 8 || p->bins > MI_MAX_BINS)
        return fail(FFDP_ERR_PARAM, "bins must be in [8, %d] (got %d)", MI_MAX_BINS, p->bins);
    if (p->hard_bins < 0 || p->hard_bins > 2) return fail(FFDP_ERR_PARAM, "hard_bins must be 0, 1 or 2");
    if (p->pad_mode != FFDP_PAD_BORDER && p->pad_mode != FFDP_PAD_ZEROS)
        return fail(FFDP_ERR_PARAM, "pad_mode must be 0 (border) or 1 (zeros)");
    if (p->check_finite != 0 && p->check_finite != 1) return fail(FFDP_ERR_PARAM, "check_finite must be 0 or 1");
    return FFDP_OK;
}

// Checked mode (check_finite = 1): the flag word is cleared and set by a pass
// over the inputs before the computation; finish_checked waits for the stream
// and reports a flagged input or a non-finite loss.
int start_checked(const float* F, const float* M, const float* u, const ffdp_grid* g, const float* grad_scale,
                  unsigned* flag, hipStream_t st)
{
    const long long N = (long long)g->D * g->H * g->W;
    hipError_t e = finite_clear_launch(flag, st);
    if (e == hipSuccess) e = finite_check_launch(F, N, flag, st);
    if (e == hipSuccess) e = finite_check_launch(M, N, flag, st);
    if (e == hipSuccess && u) e = finite_check_launch(u, 3 * N, flag, st);
    if (e == hipSuccess && grad_scale) e = finite_check_launch(grad_scale, 1, flag, st);
    return hip_status(e, "checked mode (input scan)");
}

int finish_checked(int status, const unsigned* flag, const float* loss, hipStream_t st)
{
    if (status != FFDP_OK) return status;
    unsigned hf = 0;
    float hl = 0.0f;
    hipError_t e = hipMemcpyAsync(&hf, flag, sizeof(hf), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && loss) e = hipMemcpyAsync(&hl, loss, sizeof(hl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e, "checked mode (read-back)");
    if (hf) return fail(FFDP_ERR_NONFINITE, "an input (F, M, u or grad_scale) holds a NaN or infinite value");
    if (loss && !isfinite(hl)) return fail(FFDP_ERR_NONFINITE, "the loss is not finite (%g)", (double)hl);
    return FFDP_OK;
}

int check_ptrs(const char* names, int n, ...)
{
    // names: comma-separated names of the n pointers (for the error text)
    va_list ap;
    va_start(ap, n);
    int code = FFDP_OK;
    char which[64] = "";
    for (int i = 0; i < n; ++i) {
        const void* p = va_arg(ap, const void*);
        if (code != FFDP_OK) continue;
        if (!p) code = FFDP_ERR_NULL;
        else if (misaligned(p)) code = FFDP_ERR_ALIGN;
        if (code != FFDP_OK) {
            // extract the i-th name
            const char* s = names;
            for (int k = 0; k < i && s; ++k) { s = strchr(s, ','); if (s) ++s; }
            size_t len = 0;
            while (s && s[len] && s[len] != ',' && len < sizeof(which) - 1) ++len;
            if (s) memcpy(which, s, len);
            which[len] = 0;
        }
    }
    va_end(ap);
    if (code == FFDP_ERR_NULL) return fail(code, "pointer '%s' is NULL", which);
    if (code == FFDP_ERR_ALIGN) return fail(code, "pointer '%s' is not 4-byte aligned", which);
    return FFDP_OK;
}

int check_opt_ptr(const void* p, const char* name)
{
    if (p && misaligned(p)) return fail(FFDP_ERR_ALIGN, "pointer '%s' is not 4-byte aligned", name);
    return FFDP_OK;
}

double roi_voxels(const ffdp_grid* g)
{
    return (double)(g->roi_hi[0] - g->roi_lo[0]) * (double)(g->roi_hi[1] - g->roi_lo[1]) *
           (double)(g->roi_hi[2] - g->roi_lo[2]);
}

void fill_roi(const ffdp_grid* g, int roi[6])
{
    roi[0] = (int)g->roi_lo[0]; roi[1] = (int)g->roi_hi[0];
    roi[2] = (int)g->roi_lo[1]; roi[3] = (int)g->roi_hi[1];
    roi[4] = (int)g->roi_lo[2]; roi[5] = (int)g->roi_hi[2];
}

// fused windows: one double per thread block of the largest plan over the
// modes of the window; wide windows: the FP64 fields and block partials of
// the separable passes; then 16 bytes for the checked-mode flag
size_t lncc_ws(const ffdp_grid* g, int window)
{
    if (window > LNCC_FUSED_MAX_WINDOW) return wide_ws_bytes((int)g->D, (int)g->H, (int)g->W) + 16;
    return (size_t)lncc_max_blocks((int)g->D, (int)g->H, (int)g->W, window) * sizeof(double) + 16;
}
unsigned* lncc_flag(void* ws, const ffdp_grid* g, int window)
{
    return reinterpret_cast<unsigned*>(static_cast<char*>(ws) + lncc_ws(g, window) - 16);
}

// the B^2 histogram, its NaN flag, the checked-mode flag
size_t mi_ws(const ffdp_mi_params* p) { return ((size_t)p->bins * p->bins + 2) * sizeof(unsigned long long); }
unsigned* mi_flag(void* ws, const ffdp_mi_params* p)
{
    return reinterpret_cast<unsigned*>(static_cast<unsigned long long*>(ws) + (size_t)p->bins * p->bins + 1);
}

int lncc_common(const float* F, const float* M, const float* u, const ffdp_grid* g, const ffdp_lncc_params* p,
                void* ws, size_t ws_bytes, int mode, LnccArgs& a, LnccLaunch& L)
{
    int s = check_grid(g);
    if (s) return s;
    if ((s = check_lncc(p))) return s;
    if ((s = check_ptrs("F,M", 2, (const void*)F, (const void*)M))) return s;
    if ((s = check_opt_ptr(u, "u"))) return s;
    const size_t need = lncc_ws(g, p->window);
    if (!ws || ws_bytes < need)
        return fail(FFDP_ERR_WORKSPACE, "workspace of %zu bytes required (got %zu%s)", need, ws_bytes,
                    ws ? "" : ", NULL");
    if (((uintptr_t)ws) & 7u) return fail(FFDP_ERR_ALIGN, "workspace must be 8-byte aligned");
    L = lncc_plan((int)g->D, (int)g->H, (int)g->W, p->window, mode);
    a.F = F; a.M = M; a.u = u; a.gu = nullptr; a.grad_scale = nullptr;
    a.partial = (double*)ws;
    a.D = (int)g->D; a.H = (int)g->H; a.W = (int)g->W;
    fill_roi(g, a.roi);
    a.eps = p->eps;
    a.neg_inv_nroi = (float)(-1.0 / roi_voxels(g));
    a.ntx = L.ntx; a.nty = L.nty; a.zchunk = L.zchunk; a.nblocks = L.nblocks;
    a.zspan = L.zspan;
    return FFDP_OK;
}

size_t affine_ws(const ffdp_grid* g);

// ws_kind 0: the MI histogram workspace (forward); 1: the affine partials
// (composite-sampler adjoint).
int mi_common(const float* F, const float* M, const float* u, const ffdp_grid* g, const ffdp_mi_params* p,
              void* ws, size_t ws_bytes, MiArgs& a, int ws_kind = 0)
{
    int s = check_grid(g);
    if (s) return s;
    if ((s = check_mi(p))) return s;
    if (ws_kind && p->check_finite)
        return fail(FFDP_ERR_PARAM, "check_finite is not available for the composite-sampler calls");
    if ((s = check_ptrs("F,M", 2, (const void*)F, (const void*)M))) return s;
    if ((s = check_opt_ptr(u, "u"))) return s;
    const size_t need = ws_kind ? affine_ws(g) : mi_ws(p);
    if (!ws || ws_bytes < need)
        return fail(FFDP_ERR_WORKSPACE, "workspace of %zu bytes required (got %zu%s)", need, ws_bytes,
                    ws ? "" : ", NULL");
    if (((uintptr_t)ws) & 7u) return fail(FFDP_ERR_ALIGN, "workspace must be 8-byte aligned");
    a.F = F; a.M = M; a.u = u;
    a.D = (int)g->D; a.H = (int)g->H; a.W = (int)g->W;
    fill_roi(g, a.roi);
    a.bins = p->bins;
    a.affine = 0;
    a.aff = Affine{};
    a.apart = nullptr;
    return FFDP_OK;
}

// Validated device form of the composite sampler's affine part.
int affine_from(const ffdp_affine* f, Affine& o)
{
    if (!f) return fail(FFDP_ERR_NULL, "affine is NULL");
    for (int i = 0; i < 9; ++i)
        if (!isfinite(f->A[i]) || !isfinite(f->S[i])) return fail(FFDP_ERR_PARAM, "A and S must be finite");
    for (int i = 0; i < 3; ++i)
        if (!isfinite(f->t[i])) return fail(FFDP_ERR_PARAM, "t must be finite");
    for (int i = 0; i < 9; ++i) {
        o.Am[i] = (float)((double)f->A[i] - (i % 4 == 0 ? 1.0 : 0.0));
        o.S[i] = f->S[i];
    }
    for (int i = 0; i < 3; ++i) o.t[i] = f->t[i];
    return FFDP_OK;
}

size_t affine_ws(const ffdp_grid* g) { return (size_t)12 * sizeof(double) * mi_plan((int)g->D, (int)g->H, (int)g->W).nblocks; }

int check_ws(void* ws, size_t ws_bytes, size_t need)
{
    if (!ws || ws_bytes < need)
        return fail(FFDP_ERR_WORKSPACE, "workspace of %zu bytes required (got %zu%s)", need, ws_bytes,
                    ws ? "" : ", NULL");
    if (((uintptr_t)ws) & 7u) return fail(FFDP_ERR_ALIGN, "workspace must be 8-byte aligned");
    return FFDP_OK;
}

}  // namespace

extern "C" {

int ffdp_version(void) { return 100; }

const char* ffdp_status_string(int s)
{
    switch (s) {
        case FFDP_OK: return "ok";
        case FFDP_ERR_NULL: return "null pointer";
        case FFDP_ERR_SHAPE: return "bad shape or ROI";
        case FFDP_ERR_PARAM: return "bad parameter";
        case FFDP_ERR_ALIGN: return "misaligned pointer";
        case FFDP_ERR_WORKSPACE: return "workspace missing or too small";
        case FFDP_ERR_HIP: return "HIP runtime error";
        case FFDP_ERR_NONFINITE: return "non-finite input or loss";
        default: return "unknown status";
    }
}

const char* ffdp_last_error(void) { return g_err; }

size_t ffdp_lncc_workspace_bytes(const ffdp_grid* g, const ffdp_lncc_params* p)
{
    if (!g || check_dims(g->D, g->H, g->W)) return sizeof(double);
    if (p && check_lncc(p) == FFDP_OK) return lncc_ws(g, p->window);
    size_t n = 0;  // no (valid) parameters: enough for every window
    for (int w = 3; w <= LNCC_MAX_WINDOW; w += 2) n = n > lncc_ws(g, w) ? n : lncc_ws(g, w);
    return n;
}

size_t ffdp_mi_workspace_bytes(const ffdp_grid* g, const ffdp_mi_params* p)
{
    (void)g;
    if (!p || p->bins < 8 || p->bins > MI_MAX_BINS) return sizeof(unsigned long long) * (MI_MAX_BINS * MI_MAX_BINS + 2);
    return mi_ws(p);
}

size_t ffdp_mi_state_floats(int32_t bins)
{
    if (bins < 1) bins = 1;
    return (size_t)2 * bins * bins + 2 * (size_t)bins + 16;
}

int ffdp_warp(const float* M, const float* u, const ffdp_grid* g, int32_t pad_mode, float* out, void* stream)
{
    if (!g) return fail(FFDP_ERR_NULL, "grid is NULL");
    int s = check_dims(g->D, g->H, g->W);
    if (s) return s;
    if (pad_mode != FFDP_PAD_BORDER && pad_mode != FFDP_PAD_ZEROS)
        return fail(FFDP_ERR_PARAM, "pad_mode must be 0 (border) or 1 (zeros)");
    if ((s = check_ptrs("M,out", 2, (const void*)M, (const void*)out))) return s;
    if ((s = check_opt_ptr(u, "u"))) return s;
    if (out == M) return fail(FFDP_ERR_PARAM, "out must not alias M");
    return hip_status(warp_launch(M, u, (int)g->D, (int)g->H, (int)g->W, pad_mode, out, (hipStream_t)stream),
                      "ffdp_warp");
}

int ffdp_resample(const float* src, int64_t sD, int64_t sH, int64_t sW, float* dst, int64_t dD, int64_t dH,
                  int64_t dW, int32_t channels, float value_scale, void* stream)
{
    int s;
    if ((s = check_dims(sD, sH, sW))) return s;
    if ((s = check_dims(dD, dH, dW))) return s;
    if (channels < 1 || channels > 65535) return fail(FFDP_ERR_PARAM, "channels must be in [1, 65535]");
    if (!isfinite(value_scale)) return fail(FFDP_ERR_PARAM, "value_scale must be finite");
    if ((s = check_ptrs("src,dst", 2, (const void*)src, (const void*)dst))) return s;
    const char* a0 = (const char*)src;
    const char* a1 = a0 + (size_t)channels * sD * sH * sW * sizeof(float);
    const char* b0 = (const char*)dst;
    const char* b1 = b0 + (size_t)channels * dD * dH * dW * sizeof(float);
    if (a0 < b1 && b0 < a1) return fail(FFDP_ERR_PARAM, "src and dst overlap");
    return hip_status(resample_launch(src, (int)sD, (int)sH, (int)sW, dst, (int)dD, (int)dH, (int)dW, channels,
                                      value_scale, (hipStream_t)stream),
                      "ffdp_resample");
}

int ffdp_warp_lncc_fwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                       const ffdp_lncc_params* p, float* loss, void* ws, size_t ws_bytes, void* stream)
{
    LnccArgs a;
    LnccLaunch L;
    int s = lncc_common(F, M, u, g, p, ws, ws_bytes, 0, a, L);
    if (s) return s;
    if ((s = check_ptrs("loss", 1, (const void*)loss))) return s;
    hipStream_t st = (hipStream_t)stream;
    unsigned* flag = lncc_flag(ws, g, p->window);
    if (p->check_finite && (s = start_checked(F, M, u, g, nullptr, flag, st))) return s;
    if (p->window > LNCC_FUSED_MAX_WINDOW)
        s = hip_status(lncc_wide_launch(0, p->window, p->pad_mode, a, ws, loss, roi_voxels(g), st),
                       "ffdp_warp_lncc_fwd");
    else
        s = hip_status(lncc_launch(0, p->window, p->pad_mode, L, a, loss, roi_voxels(g), st), "ffdp_warp_lncc_fwd");
    return p->check_finite ? finish_checked(s, flag, loss, st) : s;
}

int ffdp_warp_lncc_bwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                       const ffdp_lncc_params* p, const float* grad_scale, float* grad_u, float* loss, void* ws,
                       size_t ws_bytes, void* stream)
{
    LnccArgs a;
    LnccLaunch L;
    int s = lncc_common(F, M, u, g, p, ws, ws_bytes, (p && p->ants_approx) ? 2 : 1, a, L);
    if (s) return s;
    if ((s = check_ptrs("grad_u", 1, (const void*)grad_u))) return s;
    if ((s = check_opt_ptr(grad_scale, "grad_scale"))) return s;
    if ((s = check_opt_ptr(loss, "loss"))) return s;
    a.gu = grad_u;
    a.grad_scale = grad_scale;
    const int mode = p->ants_approx ? 2 : 1;
    hipStream_t st = (hipStream_t)stream;
    unsigned* flag = lncc_flag(ws, g, p->window);
    if (p->check_finite && (s = start_checked(F, M, u, g, grad_scale, flag, st))) return s;
    if (p->window > LNCC_FUSED_MAX_WINDOW)
        s = hip_status(lncc_wide_launch(mode, p->window, p->pad_mode, a, ws, loss, roi_voxels(g), st),
                       "ffdp_warp_lncc_bwd");
    else
        s = hip_status(lncc_launch(mode, p->window, p->pad_mode, L, a, loss, roi_voxels(g), st),
                       "ffdp_warp_lncc_bwd");
    return p->check_finite ? finish_checked(s, flag, loss, st) : s;
}

// Library-owned LNCC block partials for ffdp_warp_lncc_bwd_noalloc: one
// array per GPU, held until the process ends.  In host code `scratch` only
// names the symbol; its device address comes from hipGetSymbolAddress, once
// per device, and only that address is ever passed to a kernel.
static __device__ __align__(256) double scratch[FFDP_NOALLOC_MAX_BLOCKS + 2];  // + the checked-mode flag

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the device that runs `stream`, looked up
// with that device current the first time the device is seen.
int scratch_address(void* stream, double** out)
{
    int dev = 0;
    hipError_t e = hipStreamGetDevice((hipStream_t)stream, &dev);
    if (e != hipSuccess) return hip_status(e, "hipStreamGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FFDP_ERR_PARAM, "device %d beyond the %d supported", dev,
                                                   kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        if ((e = hipGetDevice(&cur)) != hipSuccess) return hip_status(e, "hipGetDevice");
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return hip_status(e, "hipSetDevice");
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) {
            hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return FFDP_OK;
}

}  // namespace

int ffdp_warp_lncc_bwd_noalloc(const float* F, const float* M, const float* u, const ffdp_grid* g,
                               const ffdp_lncc_params* p, const float* grad_scale, float* grad_u, float* loss,
                               void* stream)
{
    // everything that can be checked without the device first
    int s = check_grid(g);
    if (s) return s;
    if ((s = check_lncc(p))) return s;
    const size_t need = lncc_ws(g, p->window);
    if (need > sizeof(scratch))
        return fail(FFDP_ERR_WORKSPACE,
                    "this grid and window need %zu bytes of workspace; the library-owned scratch holds %zu", need,
                    sizeof(scratch));
    if ((s = check_ptrs("F,M,grad_u", 3, (const void*)F, (const void*)M, (const void*)grad_u))) return s;
    if ((s = check_opt_ptr(u, "u"))) return s;
    if ((s = check_opt_ptr(grad_scale, "grad_scale"))) return s;
    if ((s = check_opt_ptr(loss, "loss"))) return s;
    double* part = nullptr;
    if ((s = scratch_address(stream, &part))) return s;
    // every block writes its own partial before the finalize reads them, so
    // nothing has to be cleared between calls
    return ffdp_warp_lncc_bwd(F, M, u, g, p, grad_scale, grad_u, loss, part, sizeof(scratch), stream);
}

int ffdp_warp_mi_fwd(const float* F, const float* M, const float* u, const ffdp_grid* g, const ffdp_mi_params* p,
                     float* loss, float* mi_state, void* ws, size_t ws_bytes, void* stream)
{
    MiArgs a;
    int s = mi_common(F, M, u, g, p, ws, ws_bytes, a);
    if (s) return s;
    if ((s = check_ptrs("loss,mi_state", 2, (const void*)loss, (const void*)mi_state))) return s;
    MiLaunch L = mi_plan(a.roi[1] - a.roi[0], a.roi[3] - a.roi[2], a.roi[5] - a.roi[4]);
    a.ntx = L.ntx; a.nty = L.nty; a.zchunk = L.zchunk; a.nblocks = L.nblocks;
    hipStream_t st = (hipStream_t)stream;
    unsigned* flag = mi_flag(ws, p);
    if (p->check_finite && (s = start_checked(F, M, u, g, nullptr, flag, st))) return s;
    s = hip_status(mi_fwd_launch(a, p->hard_bins, p->pad_mode, (unsigned long long*)ws, mi_state, loss,
                                 roi_voxels(g), st),
                   "ffdp_warp_mi_fwd");
    return p->check_finite ? finish_checked(s, flag, loss, st) : s;
}

int ffdp_warp_mi_bwd(const float* F, const float* M, const float* u, const ffdp_grid* g, const ffdp_mi_params* p,
                     const float* mi_state, const float* grad_scale, float* grad_u, void* ws, size_t ws_bytes,
                     void* stream)
{
    MiArgs a;
    int s = mi_common(F, M, u, g, p, ws, ws_bytes, a);
    if (s) return s;
    if ((s = check_ptrs("mi_state,grad_u", 2, (const void*)mi_state, (const void*)grad_u))) return s;
    if ((s = check_opt_ptr(grad_scale, "grad_scale"))) return s;
    MiLaunch L = mi_plan(a.D, a.H, a.W);
    a.ntx = L.ntx; a.nty = L.nty; a.zchunk = L.zchunk; a.nblocks = L.nblocks;
    hipStream_t st = (hipStream_t)stream;
    unsigned* flag = mi_flag(ws, p);
    if (p->check_finite && (s = start_checked(F, M, u, g, grad_scale, flag, st))) return s;
    s = hip_status(mi_bwd_launch(a, p->hard_bins, p->pad_mode, mi_state, grad_scale, grad_u, roi_voxels(g), st),
                   "ffdp_warp_mi_bwd");
    return p->check_finite ? finish_checked(s, flag, nullptr, st) : s;
}

size_t ffdp_affine_workspace_bytes(const ffdp_grid* g)
{
    if (!g || g->D < 1 || g->H < 1 || g->W < 1) return 0;
    return affine_ws(g);
}

int ffdp_warp_affine(const float* M, const float* u, const ffdp_grid* g, const ffdp_affine* aff, int32_t pad_mode,
                     float* out, void* stream)
{
    if (!g) return fail(FFDP_ERR_NULL, "grid is NULL");
    int s = check_dims(g->D, g->H, g->W);
    if (s) return s;
    if (pad_mode != FFDP_PAD_BORDER && pad_mode != FFDP_PAD_ZEROS)
        return fail(FFDP_ERR_PARAM, "pad_mode must be 0 (border) or 1 (zeros)");
    if ((s = check_ptrs("M,out", 2, (const void*)M, (const void*)out))) return s;
    if ((s = check_opt_ptr(u, "u"))) return s;
    if (out == M) return fail(FFDP_ERR_PARAM, "out must not alias M");
    Affine f;
    if ((s = affine_from(aff, f))) return s;
    return hip_status(warp_affine_launch(M, u, (int)g->D, (int)g->H, (int)g->W, f, pad_mode, out,
                                         (hipStream_t)stream),
                      "ffdp_warp_affine");
}

int ffdp_warp_affine_bwd(const float* M, const float* u, const ffdp_grid* g, const ffdp_affine* aff,
                         int32_t pad_mode, const float* gout, float* grad_u, double* grad_At, void* ws,
                         size_t ws_bytes, void* stream)
{
    if (!g) return fail(FFDP_ERR_NULL, "grid is NULL");
    int s = check_dims(g->D, g->H, g->W);
    if (s) return s;
    if (pad_mode != FFDP_PAD_BORDER && pad_mode != FFDP_PAD_ZEROS)
        return fail(FFDP_ERR_PARAM, "pad_mode must be 0 (border) or 1 (zeros)");
    if ((s = check_ptrs("M,gout", 2, (const void*)M, (const void*)gout))) return s;
    if ((s = check_opt_ptr(u, "u"))) return s;
    if ((s = check_opt_ptr(grad_u, "grad_u"))) return s;
    if (!grad_At) return fail(FFDP_ERR_NULL, "grad_At is NULL");
    if (((uintptr_t)grad_At) & 7u) return fail(FFDP_ERR_ALIGN, "grad_At must be 8-byte aligned");
    if ((s = check_ws(ws, ws_bytes, affine_ws(g)))) return s;
    Affine f;
    if ((s = affine_from(aff, f))) return s;
    return hip_status(warp_affine_bwd_launch(M, u, (int)g->D, (int)g->H, (int)g->W, f, pad_mode, gout, grad_u,
                                             (double*)ws, grad_At, (hipStream_t)stream),
                      "ffdp_warp_affine_bwd");
}

int ffdp_warp_mi_affine_fwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                            const ffdp_affine* aff, const ffdp_mi_params* p, float* loss, float* mi_state, void* ws,
                            size_t ws_bytes, void* stream)
{
    MiArgs a;
    int s = mi_common(F, M, u, g, p, ws, ws_bytes, a);
    if (s) return s;
    if (p->check_finite) return fail(FFDP_ERR_PARAM, "check_finite is not available for the composite-sampler calls");
    if ((s = check_ptrs("loss,mi_state", 2, (const void*)loss, (const void*)mi_state))) return s;
    if ((s = affine_from(aff, a.aff))) return s;
    a.affine = 1;
    MiLaunch L = mi_plan(a.roi[1] - a.roi[0], a.roi[3] - a.roi[2], a.roi[5] - a.roi[4]);
    a.ntx = L.ntx; a.nty = L.nty; a.zchunk = L.zchunk; a.nblocks = L.nblocks;
    return hip_status(mi_fwd_launch(a, p->hard_bins, p->pad_mode, (unsigned long long*)ws, mi_state, loss,
                                    roi_voxels(g), (hipStream_t)stream),
                      "ffdp_warp_mi_affine_fwd");
}

int ffdp_warp_mi_affine_bwd(const float* F, const float* M, const float* u, const ffdp_grid* g,
                            const ffdp_affine* aff, const ffdp_mi_params* p, const float* mi_state,
                            const float* grad_scale, float* grad_u, double* grad_At, void* ws, size_t ws_bytes,
                            void* stream)
{
    MiArgs a;
    int s = mi_common(F, M, u, g, p, ws, ws_bytes, a, 1);
    if (s) return s;
    if ((s = check_ptrs("mi_state", 1, (const void*)mi_state))) return s;
    if ((s = check_opt_ptr(grad_scale, "grad_scale"))) return s;
    if ((s = check_opt_ptr(grad_u, "grad_u"))) return s;
    if (!grad_At) return fail(FFDP_ERR_NULL, "grad_At is NULL");
    if (((uintptr_t)grad_At) & 7u) return fail(FFDP_ERR_ALIGN, "grad_At must be 8-byte aligned");
    if ((s = affine_from(aff, a.aff))) return s;
    a.affine = 1;
    a.apart = (double*)ws;
    MiLaunch L = mi_plan(a.D, a.H, a.W);
    a.ntx = L.ntx; a.nty = L.nty; a.zchunk = L.zchunk; a.nblocks = L.nblocks;
    hipError_t e = mi_bwd_launch(a, p->hard_bins, p->pad_mode, mi_state, grad_scale, grad_u, roi_voxels(g),
                                 (hipStream_t)stream);
    if (e == hipSuccess) e = affine_reduce_launch(a.apart, a.nblocks, grad_At, (hipStream_t)stream);
    return hip_status(e, "ffdp_warp_mi_affine_bwd");
}

static int check_adam(float lr, float beta1, float beta2, float eps, int64_t step)
{
    if (step < 1) return fail(FFDP_ERR_PARAM, "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return fail(FFDP_ERR_PARAM, "betas must be in [0, 1)");
    if (!(eps > 0.0f) || !isfinite(eps) || !isfinite(lr)) return fail(FFDP_ERR_PARAM, "eps > 0, lr finite required");
    return FFDP_OK;
}

// taps exp(-t^2 / (2 sigma^2)) for |t| <= R = ceil(3 sigma), normalised in double
static int gaussian_taps(float sigma, float* w)
{
    const int R = (int)ceil(3.0 * (double)sigma);
    double tot = 0.0, e[2 * SMOOTH_MAX_R + 1];
    for (int t = -R; t <= R; ++t) tot += (e[t + R] = exp(-(double)t * t / (2.0 * (double)sigma * sigma)));
    for (int k = 0; k <= 2 * R; ++k) w[k] = (float)(e[k] / tot);
    return R;
}

static bool overlap(const void* p, const void* q, size_t bytes)
{
    const char* a = (const char*)p;
    const char* b = (const char*)q;
    return a < b + bytes && b < a + bytes;
}

int ffdp_adam_step(float* x, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                   float eps, int64_t step, void* stream)
{
    int s;
    if (n < 0) return fail(FFDP_ERR_SHAPE, "n must be >= 0");
    if (n == 0) return FFDP_OK;
    if ((s = check_ptrs("x,g,m,v", 4, (const void*)x, (const void*)g, (const void*)m, (const void*)v))) return s;
    if ((s = check_adam(lr, beta1, beta2, eps, step))) return s;
    return hip_status(adam_launch(x, g, m, v, n, lr, beta1, beta2, eps, step, (hipStream_t)stream),
                      "ffdp_adam_step");
}

int ffdp_gaussian_smooth(const float* in, float* out, int64_t D, int64_t H, int64_t W, int32_t channels, float sigma,
                         void* stream)
{
    int s;
    if ((s = check_dims(D, H, W))) return s;
    if (channels < 1 || channels > 65535) return fail(FFDP_ERR_PARAM, "channels must be in [1, 65535]");
    if (!(sigma > 0.0f && sigma <= 2.0f)) return fail(FFDP_ERR_PARAM, "sigma must be in (0, 2]");
    if ((s = check_ptrs("in,out", 2, (const void*)in, (const void*)out))) return s;
    if (overlap(in, out, (size_t)channels * D * H * W * sizeof(float))) return fail(FFDP_ERR_PARAM, "in and out overlap");
    SmoothWeights w{};
    const int R = gaussian_taps(sigma, w.w);
    return hip_status(smooth_launch(in, out, (int)D, (int)H, (int)W, channels, w, R, (hipStream_t)stream),
                      "ffdp_gaussian_smooth");
}

int ffdp_smooth_adam_step(float* x, const float* g, float* m, float* v, int64_t D, int64_t H, int64_t W,
                          int32_t channels, float sigma, float lr, float beta1, float beta2, float eps, int64_t step,
                          void* stream)
{
    int s;
    if ((s = check_dims(D, H, W))) return s;
    if (channels < 1 || channels > 65535) return fail(FFDP_ERR_PARAM, "channels must be in [1, 65535]");
    if (!(sigma > 0.0f && sigma <= 2.0f)) return fail(FFDP_ERR_PARAM, "sigma must be in (0, 2]");
    if ((s = check_ptrs("x,g,m,v", 4, (const void*)x, (const void*)g, (const void*)m, (const void*)v))) return s;
    if ((s = check_adam(lr, beta1, beta2, eps, step))) return s;
    const size_t bytes = (size_t)channels * D * H * W * sizeof(float);
    if (overlap(g, x, bytes) || overlap(g, m, bytes) || overlap(g, v, bytes) || overlap(x, m, bytes) ||
        overlap(x, v, bytes) || overlap(m, v, bytes))
        return fail(FFDP_ERR_PARAM, "x, g, m and v must not overlap");
    float taps[2 * SMOOTH_MAX_R + 1];
    const int R = gaussian_taps(sigma, taps);
    const AdamK k = adam_constants(lr, beta1, beta2, eps, step);
    return hip_status(smooth_adam_launch(x, g, m, v, (int)D, (int)H, (int)W, channels, taps, R, k,
                                         (hipStream_t)stream),
                      "ffdp_smooth_adam_step");
}

}  // extern "C"

namespace {

bool misaligned_n(const void* p, unsigned n) { return (((uintptr_t)p) & (n - 1)) != 0; }

int conv_geom(const ffdp_conv_geom* cg, ConvGeom& g, bool need_b_ptr_ok)
{
    if (!cg) return fail(FFDP_ERR_NULL, "conv geometry is NULL");
    if (cg->N < 1 || cg->Di < 1 || cg->Hi < 1 || cg->Wi < 1) return fail(FFDP_ERR_SHAPE, "N, Di, Hi, Wi must be >= 1");
    if (cg->stride != 1 && cg->stride != 2) return fail(FFDP_ERR_PARAM, "stride must be 1 or 2");
    if (cg->ups != 0 && cg->ups != 1) return fail(FFDP_ERR_PARAM, "ups must be 0 or 1");
    if (cg->Ca < 4 || cg->Ca % 4 || cg->Cb < 0 || cg->Cb % 4 || cg->Cout < 4 || cg->Cout % 4)
        return fail(FFDP_ERR_PARAM, "Ca >= 4, Cb >= 0, Cout >= 4, all multiples of 4 required");
    if (cg->Ca + cg->Cb > 192 || cg->Cout > 128) return fail(FFDP_ERR_PARAM, "Ca + Cb <= 192 and Cout <= 128 required");
    if (cg->ups && ((cg->Di | cg->Hi | cg->Wi) & 1)) return fail(FFDP_ERR_SHAPE, "ups = 1 needs even Di, Hi, Wi");
    if ((double)cg->N * cg->Di * cg->Hi * cg->Wi >= 2147483648.0)
        return fail(FFDP_ERR_SHAPE, "N Di Hi Wi must stay below 2^31 voxels");
    (void)need_b_ptr_ok;
    g.N = cg->N; g.Di = cg->Di; g.Hi = cg->Hi; g.Wi = cg->Wi;
    g.stride = cg->stride; g.ups = cg->ups;
    g.Do = (g.Di - 1) / g.stride + 1; g.Ho = (g.Hi - 1) / g.stride + 1; g.Wo = (g.Wi - 1) / g.stride + 1;
    g.Ca = cg->Ca; g.Cb = cg->Cb; g.Cout = cg->Cout;
    return FFDP_OK;
}

int bf16_ptr(const void* p, const char* name, bool required)
{
    if (!p) return required ? fail(FFDP_ERR_NULL, "pointer '%s' is NULL", name) : FFDP_OK;
    if (misaligned_n(p, 8)) return fail(FFDP_ERR_ALIGN, "pointer '%s' must be 8-byte aligned", name);
    return FFDP_OK;
}

int f32_ptr(const void* p, const char* name, bool required, unsigned align)
{
    if (!p) return required ? fail(FFDP_ERR_NULL, "pointer '%s' is NULL", name) : FFDP_OK;
    if (misaligned_n(p, align)) return fail(FFDP_ERR_ALIGN, "pointer '%s' must be %u-byte aligned", name, align);
    return FFDP_OK;
}

}  // namespace

extern "C" {

int ffdp_conv3d_fwd(const uint16_t* xa, const uint16_t* xb, const uint16_t* w, const float* bias,
                    const ffdp_conv_geom* cg, int32_t act, float slope, uint16_t* y_bf16, float* y_f32, void* stream)
{
    ConvGeom g;
    int s = conv_geom(cg, g, true);
    if (s) return s;
    if ((s = bf16_ptr(xa, "xa", true)) || (s = bf16_ptr(xb, "xb", g.Cb > 0)) || (s = bf16_ptr(w, "w", true)) ||
        (s = f32_ptr(bias, "bias", false, 4)) || (s = bf16_ptr(y_bf16, "y_bf16", false)) ||
        (s = f32_ptr(y_f32, "y_f32", false, 4)))
        return s;
    if (!y_bf16 && !y_f32) return fail(FFDP_ERR_NULL, "y_bf16 and y_f32 are both NULL");
    if (act != 0 && act != 1) return fail(FFDP_ERR_PARAM, "act must be 0 or 1");
    return hip_status(conv_fwd_launch(g, (const unsigned short*)xa, (const unsigned short*)xb,
                                      (const unsigned short*)w, bias, act, slope, (unsigned short*)y_bf16, y_f32,
                                      (hipStream_t)stream),
                      "ffdp_conv3d_fwd");
}

int ffdp_conv3d_bwd_data(const float* dy, const uint16_t* y, float slope, const uint16_t* wt,
                         const ffdp_conv_geom* cg, float* dx, int32_t accumulate, void* stream)
{
    ConvGeom g;
    int s = conv_geom(cg, g, true);
    if (s) return s;
    if ((s = f32_ptr(dy, "dy", true, 16)) || (s = bf16_ptr(y, "y", false)) || (s = bf16_ptr(wt, "wt", true)) ||
        (s = f32_ptr(dx, "dx", true, 4)))
        return s;
    if (accumulate != 0 && accumulate != 1) return fail(FFDP_ERR_PARAM, "accumulate must be 0 or 1");
    return hip_status(conv_bwd_data_launch(g, dy, (const unsigned short*)y, slope, (const unsigned short*)wt, dx,
                                           accumulate, (hipStream_t)stream),
                      "ffdp_conv3d_bwd_data");
}

int ffdp_conv3d_act_grad(const float* dy, const uint16_t* y, float slope, int64_t n, uint16_t* p, void* stream)
{
    int s;
    if (n < 0) return fail(FFDP_ERR_SHAPE, "n must be >= 0");
    if ((s = f32_ptr(dy, "dy", n > 0, 4)) || (s = f32_ptr(y, "y", false, 2)) || (s = f32_ptr(p, "p", n > 0, 2)))
        return s;
    return hip_status(act_grad_launch(dy, (const unsigned short*)y, slope, (long long)n, (unsigned short*)p,
                                      (hipStream_t)stream),
                      "ffdp_conv3d_act_grad");
}

int ffdp_conv3d_bwd_data_bf16(const uint16_t* p, const uint16_t* wt, const ffdp_conv_geom* cg, float* dx,
                              int32_t accumulate, void* stream)
{
    ConvGeom g;
    int s = conv_geom(cg, g, true);
    if (s) return s;
    if ((s = f32_ptr(p, "p", true, 16)) || (s = bf16_ptr(wt, "wt", true)) || (s = f32_ptr(dx, "dx", true, 4)))
        return s;
    if (accumulate != 0 && accumulate != 1) return fail(FFDP_ERR_PARAM, "accumulate must be 0 or 1");
    return hip_status(conv_bwd_data_p_launch(g, (const unsigned short*)p, (const unsigned short*)wt, dx, accumulate,
                                             (hipStream_t)stream),
                      "ffdp_conv3d_bwd_data_bf16");
}

size_t ffdp_conv3d_bwd_weight_workspace_bytes(const ffdp_conv_geom* cg)
{
    ConvGeom g;
    if (conv_geom(cg, g, true)) return 0;
    return (size_t)conv_wgrad_plan(g).part_floats * sizeof(float);
}

int ffdp_conv3d_bwd_weight(const uint16_t* xa, const uint16_t* xb, const float* dy, const uint16_t* y, float slope,
                           const ffdp_conv_geom* cg, float* dw, float* db, void* ws, size_t ws_bytes, void* stream)
{
    ConvGeom g;
    int s = conv_geom(cg, g, true);
    if (s) return s;
    if ((s = bf16_ptr(xa, "xa", true)) || (s = bf16_ptr(xb, "xb", g.Cb > 0)) || (s = f32_ptr(dy, "dy", true, 4)) ||
        (s = bf16_ptr(y, "y", false)) || (s = f32_ptr(dw, "dw", true, 4)) || (s = f32_ptr(db, "db", false, 4)))
        return s;
    const size_t need = (size_t)conv_wgrad_plan(g).part_floats * sizeof(float);
    if (!ws || ws_bytes < need) return fail(FFDP_ERR_WORKSPACE, "workspace of %zu bytes required (got %zu)", need, ws_bytes);
    if (misaligned_n(ws, 4)) return fail(FFDP_ERR_ALIGN, "workspace must be 4-byte aligned");
    return hip_status(conv_bwd_weight_launch(g, (const unsigned short*)xa, (const unsigned short*)xb, dy,
                                             (const unsigned short*)y, slope, dw, db, (float*)ws, (hipStream_t)stream),
                      "ffdp_conv3d_bwd_weight");
}

int ffdp_conv3d_bwd_weight_bf16(const uint16_t* xa, const uint16_t* xb, const uint16_t* p, const ffdp_conv_geom* cg,
                                float* dw, float* db, void* ws, size_t ws_bytes, void* stream)
{
    ConvGeom g;
    int s = conv_geom(cg, g, true);
    if (s) return s;
    if ((s = bf16_ptr(xa, "xa", true)) || (s = bf16_ptr(xb, "xb", g.Cb > 0)) || (s = bf16_ptr(p, "p", true)) ||
        (s = f32_ptr(dw, "dw", true, 4)) || (s = f32_ptr(db, "db", false, 4)))
        return s;
    const size_t need = (size_t)conv_wgrad_plan(g).part_floats * sizeof(float);
    if (!ws || ws_bytes < need) return fail(FFDP_ERR_WORKSPACE, "workspace of %zu bytes required (got %zu)", need, ws_bytes);
    if (misaligned_n(ws, 4)) return fail(FFDP_ERR_ALIGN, "workspace must be 4-byte aligned");
    return hip_status(conv_bwd_weight_p_launch(g, (const unsigned short*)xa, (const unsigned short*)xb,
                                               (const unsigned short*)p, dw, db, (float*)ws, (hipStream_t)stream),
                      "ffdp_conv3d_bwd_weight_bf16");
}

int ffdp_conv3d_weight_prep(const float* w, int32_t Cout, int32_t Cin, uint16_t* w_bf16, uint16_t* wt_bf16,
                            void* stream)
{
    int s;
    if (Cout < 1 || Cin < 1 || Cout > 4096 || Cin > 4096) return fail(FFDP_ERR_SHAPE, "Cout, Cin must be in [1, 4096]");
    if ((s = f32_ptr(w, "w", true, 4)) || (s = bf16_ptr(w_bf16, "w_bf16", false)) ||
        (s = bf16_ptr(wt_bf16, "wt_bf16", false)))
        return s;
    return hip_status(weight_prep_launch(w, Cout, Cin, (unsigned short*)w_bf16, (unsigned short*)wt_bf16,
                                         (hipStream_t)stream),
                      "ffdp_conv3d_weight_prep");
}

int ffdp_unet_pack_pair(const float* F, const float* M, int64_t nvox, uint16_t* x, void* stream)
{
    int s;
    if (nvox < 1) return fail(FFDP_ERR_SHAPE, "nvox must be >= 1");
    if ((s = f32_ptr(F, "F", true, 4)) || (s = f32_ptr(M, "M", true, 4)) || (s = bf16_ptr(x, "x", true))) return s;
    return hip_status(pack_pair_launch(F, M, nvox, (unsigned short*)x, (hipStream_t)stream), "ffdp_unet_pack_pair");
}

int ffdp_concat_grad_split(const float* dxcat, const ffdp_conv_geom* cg, float* dxa, float* dxb, int32_t acc_a,
                           int32_t acc_b, void* stream)
{
    ConvGeom g;
    int s = conv_geom(cg, g, true);
    if (s) return s;
    if (!g.ups) return fail(FFDP_ERR_PARAM, "ffdp_concat_grad_split needs ups = 1");
    if ((s = f32_ptr(dxcat, "dxcat", true, 16)) || (s = f32_ptr(dxa, "dxa", true, 16)) ||
        (s = f32_ptr(dxb, "dxb", g.Cb > 0, 16)))
        return s;
    return hip_status(split_grad_launch(g, dxcat, dxa, dxb, acc_a ? 1 : 0, acc_b ? 1 : 0, (hipStream_t)stream),
                      "ffdp_concat_grad_split");
}

size_t ffdp_mse_workspace_bytes(void) { return (size_t)MSE_BLOCKS * sizeof(double); }

int ffdp_mse_disp(const float* pred, int32_t Cp, const float* target, int64_t nvox, int32_t N, float* dpred,
                  float* loss, void* ws, size_t ws_bytes, void* stream)
{
    int s;
    if (Cp < 3 || N < 1 || nvox < 1) return fail(FFDP_ERR_SHAPE, "Cp >= 3, N >= 1, nvox >= 1 required");
    if ((s = f32_ptr(pred, "pred", true, 4)) || (s = f32_ptr(target, "target", true, 4)) ||
        (s = f32_ptr(dpred, "dpred", false, 4)) || (s = f32_ptr(loss, "loss", false, 4)))
        return s;
    if (!ws || ws_bytes < (size_t)MSE_BLOCKS * sizeof(double) || misaligned_n(ws, 8))
        return fail(FFDP_ERR_WORKSPACE, "workspace of %zu 8-byte aligned bytes required", (size_t)MSE_BLOCKS * 8);
    return hip_status(mse_launch(pred, Cp, target, nvox, N, dpred, (double*)ws, MSE_BLOCKS, loss, (hipStream_t)stream),
                      "ffdp_mse_disp");
}

int ffdp_unpack_disp(const float* pred, int32_t Cp, int64_t nvox, int32_t N, float* u, void* stream)
{
    int s;
    if (Cp < 3 || N < 1 || nvox < 1) return fail(FFDP_ERR_SHAPE, "Cp >= 3, N >= 1, nvox >= 1 required");
    if ((s = f32_ptr(pred, "pred", true, 4)) || (s = f32_ptr(u, "u", true, 4))) return s;
    return hip_status(unpack_disp_launch(pred, Cp, nvox, N, u, (hipStream_t)stream), "ffdp_unpack_disp");
}

}  // extern "C"
