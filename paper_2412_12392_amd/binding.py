"""Python binding of libm3s over torch device tensors.

Marshals torch tensors (device memory) and the current HIP stream into the C
ABI of include/m3s.h.  Every step of the matcher runs inside libm3s's HIP
kernels; nothing here computes.  There is no CPU fallback: a missing library
or a CPU tensor raises.

    res = match(Xii, Xji, Dii, Dji, Qii, Qji)        # MASt3R-SLAM Sec. 3.2
    gXii, gXji = match_backward(Xii, Xji, res.p, res.valid, grad_p, grad_xhat)
    outs = match_batched([EdgeInput(...), ...], graph=True)
    p, xhat, idx, valid, theta = MatchFunction.apply(Xii, Xji, Dii, Dji, Qii, Qji, None, params)
    T, info = track_pose(Xk, Xf, idx, valid, Qf, Qk, T)   # Sec. 3.3, T updated in place
    fuse_pointmap(Xc, Cc, X, C, T)                           # Eq. 8, in place
    T_WC, info = backend_gn(Xc_all, Q_all, edges, idx_all, valid_all, T_WC)   # Sec. 3.5
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib


@dataclass
class MatchResult:
    p: torch.Tensor                  # (H, W, 2) float32, continuous match p*
    idx: torch.Tensor                # (H, W) int32, refined linear index or -1
    valid: torch.Tensor              # (H, W) uint8
    theta: Optional[torch.Tensor]    # (H, W) float32 residual angle, or None
    xhat: Optional[torch.Tensor]     # (H, W, 3) float32 X^i_i at p*, or None


@dataclass
class EdgeInput:
    Xii: torch.Tensor
    Xji: torch.Tensor
    Dii: torch.Tensor
    Dji: torch.Tensor
    Qii: Optional[torch.Tensor] = None
    Qji: Optional[torch.Tensor] = None
    p_init: Optional[torch.Tensor] = None
    max_iter: int = -1               # < 0: the common value
    refine_radius: int = -1


def params(**overrides) -> _lib.Params:
    """Matching parameters: library defaults (K 10, lambda 1e-8, r 3, q_min 1.5,
    max_theta 1e-4, no distance gate) with keyword overrides."""
    return _lib.default_params(None, **overrides)


def _ptr(t: Optional[torch.Tensor], dtype=torch.float32, shape=None) -> int:
    if t is None:
        return 0
    if not t.is_cuda:
        raise ValueError("libm3s takes device tensors (got a CPU tensor)")
    if t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(t.shape)))
    return t.data_ptr()


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


_ws_cache: dict = {}
_WS_CACHE_STREAMS = 16


def _workspace(nbytes: int, device, stream=None) -> torch.Tensor:
    """Device workspace of at least nbytes for one call on `stream` (torch
    allocations are >= 256-byte aligned).

    Outside a graph capture, one buffer per (device, stream) is kept and grown
    as needed: the calls of one stream run in order, so they may share it, and
    calls on different streams never do.  The buffer is allocated with its
    stream current, so when it is dropped the allocator reuses its memory only
    in that stream's order.  During a torch graph capture every call gets a
    buffer of its own from the capture's memory pool, which torch keeps for
    the graph's lifetime, and it is never cached: later eager calls cannot
    overwrite what a replay reads.
    """
    s = torch.cuda.current_stream(device) if stream is None else stream
    if torch.cuda.is_current_stream_capturing():
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    key = (torch.device(device).index, s.cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        with torch.cuda.stream(s):
            buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache.pop(key, None)
        _ws_cache[key] = buf
        while len(_ws_cache) > _WS_CACHE_STREAMS:
            _ws_cache.pop(next(iter(_ws_cache)))
    return buf


def _pair(Xii, Xji, Dii=None, Dji=None, Qii=None, Qji=None, p_init=None) -> _lib.Pair:
    H, W = Xii.shape[:2]
    D = Dii.shape[2] if Dii is not None else 0
    return _lib.Pair(H, W, D, _ptr(Xii, shape=(H, W, 3)), _ptr(Xji, shape=(H, W, 3)),
                     _ptr(Dii, shape=(H, W, D)), _ptr(Dji, shape=(H, W, D)),
                     _ptr(Qii, shape=(H, W)), _ptr(Qji, shape=(H, W)), _ptr(p_init, shape=(H, W, 2)))


def _alloc_outputs(H, W, device, want_theta, want_xhat):
    p = torch.empty((H, W, 2), dtype=torch.float32, device=device)
    idx = torch.empty((H, W), dtype=torch.int32, device=device)
    valid = torch.empty((H, W), dtype=torch.uint8, device=device)
    theta = torch.empty((H, W), dtype=torch.float32, device=device) if want_theta else None
    xhat = torch.empty((H, W, 3), dtype=torch.float32, device=device) if want_xhat else None
    return MatchResult(p, idx, valid, theta, xhat)


def _outputs(res: MatchResult) -> _lib.Outputs:
    return _lib.Outputs(_ptr(res.p), _ptr(res.idx, torch.int32), _ptr(res.valid, torch.uint8),
                        _ptr(res.theta), _ptr(res.xhat))


def match(Xii, Xji, Dii, Dji, Qii=None, Qji=None, p_init=None, prm: Optional[_lib.Params] = None,
          want_theta: bool = True, want_xhat: bool = False, out: Optional[MatchResult] = None,
          stream=None) -> MatchResult:
    """m3s_match_fwd on one pair of (H, W, 3) pointmaps and (H, W, D) descriptors."""
    lib = _lib.load()
    H, W = Xii.shape[:2]
    pair = _pair(Xii, Xji, Dii, Dji, Qii, Qji, p_init)
    prm = prm if prm is not None else params()
    res = out if out is not None else _alloc_outputs(H, W, Xii.device, want_theta, want_xhat)
    o = _outputs(res)
    nbytes = lib.m3s_workspace_bytes(ctypes.byref(pair), ctypes.byref(prm))
    ws = _workspace(nbytes, Xii.device, stream)
    st = lib.m3s_match_fwd(ctypes.byref(pair), ctypes.byref(prm), ctypes.byref(o), ws.data_ptr(), ws.numel(),
                           _stream(stream))
    _lib.check(lib, "m3s_match_fwd", st)
    return res


def match_noalloc(Xii, Xji, Dii, Dji, Qii=None, Qji=None, p_init=None, prm: Optional[_lib.Params] = None,
                  *, out: MatchResult, stream=None) -> MatchResult:
    """m3s_match_fwd_noalloc: the forward with the library's static device scratch
    (H * W <= M3S_NOALLOC_MAX_PIXELS) into the caller's outputs `out`; neither
    this call nor the library allocates memory."""
    lib = _lib.load()
    pair = _pair(Xii, Xji, Dii, Dji, Qii, Qji, p_init)
    prm = prm if prm is not None else params()
    o = _outputs(out)
    st = lib.m3s_match_fwd_noalloc(ctypes.byref(pair), ctypes.byref(prm), ctypes.byref(o), _stream(stream))
    _lib.check(lib, "m3s_match_fwd_noalloc", st)
    return out


def match_backward(Xii, Xji, p, valid, grad_p, grad_xhat=None, stream=None):
    """m3s_match_bwd: (dL/dXii, dL/dXji) through p* and xhat."""
    lib = _lib.load()
    H, W = Xii.shape[:2]
    pair = _pair(Xii, Xji)
    fwd = _lib.Outputs(_ptr(p, shape=(H, W, 2)), 0, _ptr(valid, torch.uint8, shape=(H, W)), 0, 0)
    gXii = torch.empty((H, W, 3), dtype=torch.float32, device=Xii.device)
    gXji = torch.empty((H, W, 3), dtype=torch.float32, device=Xii.device)
    st = lib.m3s_match_bwd(ctypes.byref(pair), ctypes.byref(fwd), _ptr(grad_p, shape=(H, W, 2)),
                           _ptr(grad_xhat, shape=(H, W, 3)), _ptr(gXii), _ptr(gXji), _stream(stream))
    _lib.check(lib, "m3s_match_bwd", st)
    return gXii, gXji


@dataclass
class BwdEdgeInput:
    Xii: torch.Tensor                 # (H, W, 3)
    Xji: torch.Tensor                 # (H, W, 3)
    p: torch.Tensor                   # (H, W, 2) forward p*
    valid: torch.Tensor               # (H, W) uint8
    grad_p: torch.Tensor              # (H, W, 2)
    grad_xhat: Optional[torch.Tensor] = None   # (H, W, 3)


def make_bwd_edges(inputs: Sequence[BwdEdgeInput], outs=None):
    """Host backward edge table plus freshly allocated (or given) (grad_Xii, grad_Xji) per edge."""
    n = len(inputs)
    table = (_lib.BwdEdge * n)()
    grads = []
    for k, e in enumerate(inputs):
        H, W = e.Xii.shape[:2]
        if outs is not None:
            gi, gj = outs[k]
        else:
            gi = torch.empty((H, W, 3), dtype=torch.float32, device=e.Xii.device)
            gj = torch.empty((H, W, 3), dtype=torch.float32, device=e.Xii.device)
        table[k] = _lib.BwdEdge(H, W, _ptr(e.Xii, shape=(H, W, 3)), _ptr(e.Xji, shape=(H, W, 3)),
                                _ptr(e.p, shape=(H, W, 2)), _ptr(e.valid, torch.uint8, shape=(H, W)),
                                _ptr(e.grad_p, shape=(H, W, 2)), _ptr(e.grad_xhat, shape=(H, W, 3)),
                                _ptr(gi, shape=(H, W, 3)), _ptr(gj, shape=(H, W, 3)))
        grads.append((gi, gj))
    return table, grads


def match_backward_batched(inputs: Sequence[BwdEdgeInput], graph: bool = True, outs=None, stream=None,
                           accumulate: bool = False):
    """m3s_match_bwd_batched: the implicit adjoint of every edge in one persistent launch
    (after one launch that zeroes every grad_Xii, or, with accumulate, added to the
    given grad_Xii's contents); returns [(grad_Xii, grad_Xji)] per edge."""
    lib = _lib.load()
    if accumulate and outs is None:
        raise ValueError("accumulate needs the grad_Xii buffers (outs) to add to")
    table, grads = make_bwd_edges(inputs, outs)
    n = len(inputs)
    nbytes = lib.m3s_bwd_batched_workspace_bytes(n)
    ws = _workspace(nbytes, inputs[0].Xii.device, stream)
    flags = (_lib.M3S_BATCH_GRAPH if graph else 0) | (_lib.M3S_BWD_ACCUMULATE if accumulate else 0)
    st = lib.m3s_match_bwd_batched(table, n, flags, ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(lib, "m3s_match_bwd_batched", st)
    return grads


def make_edges(inputs: Sequence[EdgeInput], want_theta=True, want_xhat=False, outs=None):
    """Host edge table plus freshly allocated (or given) outputs."""
    n = len(inputs)
    table = (_lib.Edge * n)()
    results = []
    for k, e in enumerate(inputs):
        H, W = e.Xii.shape[:2]
        res = outs[k] if outs is not None else _alloc_outputs(H, W, e.Xii.device, want_theta, want_xhat)
        table[k].in_ = _pair(e.Xii, e.Xji, e.Dii, e.Dji, e.Qii, e.Qji, e.p_init)
        table[k].out = _outputs(res)
        table[k].max_iter = e.max_iter
        table[k].refine_radius = e.refine_radius
        results.append(res)
    return table, results


def match_batched(inputs: Sequence[EdgeInput], prm: Optional[_lib.Params] = None, graph: bool = True,
                  autotune: bool = False, want_theta=True, want_xhat=False, outs=None, stream=None):
    """m3s_match_batched: every edge in one persistent launch; returns one MatchResult per edge."""
    lib = _lib.load()
    prm = prm if prm is not None else params()
    table, results = make_edges(inputs, want_theta, want_xhat, outs)
    n = len(inputs)
    nbytes = lib.m3s_batched_workspace_bytes(table, n, ctypes.byref(prm))
    if nbytes == 0:
        raise _lib.M3SError("m3s_batched_workspace_bytes", _lib.M3S_OK + 2, "invalid edges")
    ws = _workspace(nbytes, inputs[0].Xii.device, stream)
    flags = (_lib.M3S_BATCH_GRAPH if graph else 0) | (_lib.M3S_BATCH_AUTOTUNE if autotune else 0)
    st = lib.m3s_match_batched(table, n, ctypes.byref(prm), flags, ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(lib, "m3s_match_batched", st)
    return results


def match_stats(res: MatchResult, stream=None) -> torch.Tensor:
    """m3s_match_stats: device int32 tensor [valid count, distinct matched reference pixels]."""
    lib = _lib.load()
    H, W = res.idx.shape
    fwd = _lib.Outputs(0, _ptr(res.idx, torch.int32, shape=(H, W)), _ptr(res.valid, torch.uint8, shape=(H, W)), 0, 0)
    counts = torch.empty(2, dtype=torch.int32, device=res.idx.device)
    nbytes = lib.m3s_stats_workspace_bytes(H, W)
    ws = _workspace(nbytes, res.idx.device, stream)
    st = lib.m3s_match_stats(ctypes.byref(fwd), H, W, _ptr(counts, torch.int32), ws.data_ptr(), ws.numel(),
                             _stream(stream))
    _lib.check(lib, "m3s_match_stats", st)
    return counts


def track_params(**overrides) -> _lib.TrackParams:
    """Tracking parameters: library defaults (10 iterations, q_min 1.5, sigma_ray 0.003,
    sigma_dist 0.1, Huber 1.345) with keyword overrides."""
    return _lib.default_track_params(None, **overrides)


def track_pose(Xk, Xf, idx, valid, Qf, Qk, T, prm: Optional[_lib.TrackParams] = None, stream=None):
    """m3s_track_pose (Sec. 3.3): refines the Sim(3) pose T (device float32 (3, 4), updated in
    place) from the matches idx/valid of the keyframe's pixels.  Returns (T, info) with info the
    device float32 tensor [cost, matches used, iterations solved, last step norm]."""
    lib = _lib.load()
    H, W = Xk.shape[:2]
    prob = _lib.TrackProblem(H, W, _ptr(Xk, shape=(H, W, 3)), _ptr(Xf, shape=(H, W, 3)),
                             _ptr(idx, torch.int32, shape=(H, W)), _ptr(valid, torch.uint8, shape=(H, W)),
                             _ptr(Qf, shape=(H, W)), _ptr(Qk, shape=(H, W)))
    prm = prm if prm is not None else track_params()
    info = torch.empty(4, dtype=torch.float32, device=Xk.device)
    nbytes = lib.m3s_track_workspace_bytes(H, W)
    ws = _workspace(nbytes, Xk.device, stream)
    st = lib.m3s_track_pose(ctypes.byref(prob), ctypes.byref(prm), _ptr(T, shape=(3, 4)), _ptr(info), ws.data_ptr(),
                            ws.numel(), _stream(stream))
    _lib.check(lib, "m3s_track_pose", st)
    return T, info


def fuse_pointmap(Xc, Cc, X, C, T, stream=None):
    """m3s_fuse_pointmap (Sec. 3.3, Eq. 8): updates the canonical pointmap Xc (H, W, 3) and its
    confidence Cc (H, W) in place from the frame's prediction X, C and the device pose T (3, 4)."""
    lib = _lib.load()
    H, W = Xc.shape[:2]
    prob = _lib.FuseProblem(H, W, _ptr(Xc, shape=(H, W, 3)), _ptr(Cc, shape=(H, W)), _ptr(X, shape=(H, W, 3)),
                            _ptr(C, shape=(H, W)))
    st = lib.m3s_fuse_pointmap(ctypes.byref(prob), _ptr(T, shape=(3, 4)), _stream(stream))
    _lib.check(lib, "m3s_fuse_pointmap", st)
    return Xc, Cc


def backend_params(**overrides) -> _lib.BackendParams:
    """Backend parameters: library defaults (10 iterations, q_min 1.5, sigma_ray 0.003,
    sigma_dist 0.1, Huber 1.345, step_tol 0) with keyword overrides."""
    return _lib.default_backend_params(None, **overrides)


def backend_gn(Xc, Q, edges, idx, valid, T_WC, prm: Optional[_lib.BackendParams] = None, stream=None):
    """m3s_backend_gn (Sec. 3.5): refines the world poses T_WC (device float32 (N, 3, 4), updated in
    place, keyframe 0 held) over the edges (device int32 (E, 2)) with matches idx/valid (E, H, W).
    Returns (T_WC, info) with info the device float32 tensor [cost, matches used, steps applied,
    last step norm]."""
    lib = _lib.load()
    N, H, W = Xc.shape[:3]
    E = edges.shape[0]
    prob = _lib.BackendProblem(N, H, W, E, _ptr(Xc, shape=(N, H, W, 3)), _ptr(Q, shape=(N, H, W)),
                               _ptr(edges, torch.int32, shape=(E, 2)), _ptr(idx, torch.int32, shape=(E, H, W)),
                               _ptr(valid, torch.uint8, shape=(E, H, W)))
    prm = prm if prm is not None else backend_params()
    info = torch.empty(4, dtype=torch.float32, device=Xc.device)
    nbytes = lib.m3s_backend_workspace_bytes(N, H, W, E)
    ws = _workspace(nbytes, Xc.device, stream)
    st = lib.m3s_backend_gn(ctypes.byref(prob), ctypes.byref(prm), _ptr(T_WC, shape=(N, 3, 4)), _ptr(info),
                            ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(lib, "m3s_backend_gn", st)
    return T_WC, info


def set_launch(tile_config: int = -1, grid: int = -1, xcd_remap: int = -1, ray_margin: int = -1,
               lm_unroll: int = -1):
    """m3s_debug_set_launch for the calling thread (all -1: the library's choice)."""
    lib = _lib.load()
    if tile_config < 0 and grid <= 0 and xcd_remap < 0 and ray_margin <= 0 and lm_unroll <= 0:
        lib.m3s_debug_set_launch(None)
    else:
        cfg = _lib.LaunchConfig(tile_config, grid, xcd_remap, ray_margin, lm_unroll)
        lib.m3s_debug_set_launch(ctypes.byref(cfg))


def last_batched_launch() -> dict:
    """m3s_batched_last_launch: the launch the calling thread's last batched call used."""
    lib = _lib.load()
    cfg = _lib.LaunchConfig()
    lib.m3s_batched_last_launch(ctypes.byref(cfg))
    return dict(tile_config=cfg.tile_config, grid=cfg.grid, ray_margin=cfg.ray_margin, lm_unroll=cfg.lm_unroll)


def set_tune_cache(path: Optional[str]):
    """m3s_set_tune_cache: load and from now on update the on-disk autotuning cache (None: stop writing)."""
    lib = _lib.load()
    _lib.check(lib, "m3s_set_tune_cache", lib.m3s_set_tune_cache(None if path is None else path.encode()))


def path_counters(reset: bool = False) -> dict:
    """m3s_path_counters: fallback paths taken on the current device since the last reset."""
    lib = _lib.load()
    buf = (ctypes.c_int64 * _lib.M3S_PATH_COUNTERS)()
    _lib.check(lib, "m3s_path_counters", lib.m3s_path_counters(buf, 1 if reset else 0))
    return {name: int(buf[k]) for k, name in enumerate(_lib.PATH_NAMES)}


def last_batched_config():
    lib = _lib.load()
    g, t = ctypes.c_int32(), ctypes.c_int32()
    lib.m3s_batched_last_config(ctypes.byref(g), ctypes.byref(t))
    return g.value, t.value


class MatchFunction(torch.autograd.Function):
    """Differentiable matcher: (Xii, Xji, ...) -> (p, xhat, idx, valid, theta).

    Gradients reach Xii and Xji through the continuous match p* and the
    sampled point xhat (implicit adjoint, m3s_match_bwd).  idx, valid and
    theta are not differentiable, and descriptors, confidences and p_init get
    no gradient (the refine offset is piecewise constant).
    """

    @staticmethod
    def forward(ctx, Xii, Xji, Dii, Dji, Qii=None, Qji=None, p_init=None, prm=None):
        Xii_c, Xji_c = Xii.contiguous(), Xji.contiguous()
        res = match(Xii_c, Xji_c, Dii.contiguous(), Dji.contiguous(),
                    None if Qii is None else Qii.contiguous(), None if Qji is None else Qji.contiguous(),
                    None if p_init is None else p_init.contiguous(), prm, want_theta=True, want_xhat=True)
        ctx.save_for_backward(Xii_c, Xji_c, res.p, res.valid)
        ctx.mark_non_differentiable(res.idx, res.valid, res.theta)
        return res.p, res.xhat, res.idx, res.valid, res.theta

    @staticmethod
    def backward(ctx, grad_p, grad_xhat, _gi, _gv, _gt):
        Xii, Xji, p, valid = ctx.saved_tensors
        if grad_p is None:
            grad_p = torch.zeros_like(p)
        gXii, gXji = match_backward(Xii, Xji, p, valid, grad_p.contiguous(),
                                    None if grad_xhat is None else grad_xhat.contiguous())
        return gXii, gXji, None, None, None, None, None, None
