"""FP64 CPU oracle of the fused warp + dissimilarity path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU timing leg import
this package.  It shares no code with the library's HIP path.
"""
from .oracle import (  # noqa: F401
    adam, conv3d_bwd_data, conv3d_bwd_weight, conv3d_fwd, gaussian_smooth, lncc, lncc_grad_u_at, lncc_loss_mw, load,
    max_threads, mi, mi_affine, mi_grad_u_at, mi_pmf, parzen, resample, set_threads, warp, warp_affine, warp_affine_bwd,
)
