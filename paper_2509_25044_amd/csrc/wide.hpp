// Host-side declarations of the wide-window LNCC passes (lncc_wide.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "internal.hpp"

namespace ffdp {

// Windows 3..9 run the fused kernel; 11..15 the separable FP64 passes, whose
// workspace holds 8 N doubles (the xy sums of the five products, later of
// a, c, e; the fields a, c, e) and then the block partials of the loss.
constexpr int LNCC_FUSED_MAX_WINDOW = 9;
constexpr int LNCC_MAX_WINDOW = 15;

struct WidePlan {
    int ncx, ncy, zchunk, nchunks, nblocks;
};
WidePlan wide_plan(int D, int H, int W);
size_t wide_ws_bytes(int D, int H, int W);
// mode as lncc_launch; a.partial and the plan fields of a are not used; ws
// holds wide_ws_bytes(D, H, W), 8-byte aligned.
hipError_t lncc_wide_launch(int mode, int win, int pad, const LnccArgs& a, void* ws, float* loss, double nroi,
                            hipStream_t st);

}  // namespace ffdp
