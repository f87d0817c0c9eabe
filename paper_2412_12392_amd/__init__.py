"""MI355X-native projective pointmap matching (MASt3R-SLAM, arXiv 2412.12392, Sec. 3.2)
and the consumers of its matches: tracking pose solve and pointmap fusion (Sec. 3.3),
backend pose-graph Gauss-Newton (Sec. 3.5).

Everything runs in libm3s.so: hand-written HIP kernels for gfx950 behind the C
ABI of include/m3s.h.  This package is its thin Python binding over torch device
tensors.  Build the library with ``python -m paper_2412_12392_amd.build``.
"""
from .binding import (BwdEdgeInput, EdgeInput, MatchFunction, MatchResult, backend_gn,  # noqa: F401
                      backend_params, fuse_pointmap, last_batched_config, last_batched_launch, make_bwd_edges, make_edges, match,
                      match_backward, match_backward_batched, match_batched, match_noalloc, match_stats, params,
                      path_counters, set_launch, set_tune_cache, track_params, track_pose)
from ._lib import M3SError, load as load_library  # noqa: F401
