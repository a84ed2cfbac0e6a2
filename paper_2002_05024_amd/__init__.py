"""MI355X-native Schur reduction (small-bulge multishift QR with aggressive early
deflation) for real upper Hessenberg matrices.

The numerical work happens in ``libneig.so`` (hand-written HIP for gfx950, C ABI
declared in ``include/neig.h``); :mod:`paper_2002_05024_amd.binding` marshals
torch tensors (device memory, current stream) into those calls.  Importing this
package does not load the library; the first call does, and raises if it is
missing.
"""
from .binding import (  # noqa: F401
    NeigError,
    library_path,
    load_library,
    schur,
    schur_batched,
    batched_tables,
    launch_batched,
    set_batched_tune,
    get_batched_tune,
    set_params,
    get_params,
    get_stats,
    sweep,
    aed,
    small_schur,
    reorder,
    hessenberg,
    finalize,
    policy_bins,
    policy_set,
    policy_log,
    policy_features,
    mlp_grad,
    mlp_adam,
    mlp_infer,
)
