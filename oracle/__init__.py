"""FP64 CPU oracle for iterative projective pointmap matching (test infrastructure).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python binding)
never imports, links or calls anything here.

The arithmetic lives in ``m3s_oracle.c`` (plain C, double precision, one query
pixel at a time, OpenMP over queries); this module compiles it with gcc when no
build exists and marshals numpy arrays through ctypes.  ``unrolled.py`` is an
independent vectorised fp64 torch-CPU restatement used to cross-check the
backward by differentiating through the unrolled iterations.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "m3s_oracle.c")
_TRACK_SRC = os.path.join(_HERE, "m3s_track_oracle.c")
_BACKEND_SRC = os.path.join(_HERE, "m3s_backend_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_m3s.so")

# Defaults of the matching workloads: 10 LM iterations, lambda 1e-8, refine
# radius 3, confidence gate 1.5, residual-angle gate 1e-4 rad, 3D gate off.
DEFAULTS = dict(K=10, lambda0=1e-8, r=3, levels=1, conf_min=1.5, max_theta=1e-4, max_dist=math.inf)


def compile_oracle(src: str = _SRC, out: str = _LIB_PATH, extra_flags=(), track_src: str = _TRACK_SRC,
                   backend_src: str = _BACKEND_SRC) -> str:
    """Compile the C oracle (matching, tracking and backend sources) into a shared library (gcc, -O2, OpenMP)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", *extra_flags, src, track_src, backend_src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None


def load(path: str | None = None):
    """Load (building first if absent) the oracle library; returns the ctypes handle."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        newest = max(os.path.getmtime(f) for f in (_SRC, _TRACK_SRC, _BACKEND_SRC))
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < newest:
            compile_oracle()
        _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def _declare(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    up = ctypes.POINTER(ctypes.c_uint8)
    c_int, c_long, c_double = ctypes.c_int, ctypes.c_long, ctypes.c_double
    lib.oracle_match_fwd.argtypes = [c_int, c_int, c_int, dp, dp, dp, dp, dp, dp, dp,
                                     c_int, c_double, c_int, c_int, c_double, c_double, c_double,
                                     dp, ip, up, dp, dp, dp, c_int]
    lib.oracle_match_fwd.restype = c_int
    lib.oracle_cost_grid.argtypes = [c_int, c_int, dp, dp, c_long, dp, dp, dp]
    lib.oracle_cost_grid.restype = c_int
    lib.oracle_ray_images.argtypes = [c_int, c_int, dp, dp, dp, dp]
    lib.oracle_ray_images.restype = c_int
    lib.oracle_match_bwd.argtypes = [c_int, c_int, dp, dp, dp, up, dp, dp, dp, dp]
    lib.oracle_match_bwd.restype = c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = c_int
    lp = ctypes.POINTER(ctypes.c_long)
    lib.oracle_track_pose.argtypes = [c_int, c_int, dp, dp, ip, up, dp, dp, c_double, c_double, c_double, c_double,
                                      c_int, dp, dp, lp, dp, dp]
    lib.oracle_track_pose.restype = c_int
    lib.oracle_sim3_exp.argtypes = [dp, dp]
    lib.oracle_sim3_exp.restype = None
    lib.oracle_track_residual.argtypes = [dp, dp, dp, dp, dp]
    lib.oracle_track_residual.restype = None
    lib.oracle_fuse.argtypes = [ctypes.c_long, dp, dp, dp, dp, dp]
    lib.oracle_fuse.restype = None
    lib.oracle_backend_residual.argtypes = [dp, dp, dp, dp, dp, dp, dp]
    lib.oracle_backend_residual.restype = c_int
    lib.oracle_backend_gn.argtypes = [c_int, c_int, c_int, dp, dp, c_int, ip, ip, ip, up, c_double, c_double,
                                      c_double, c_double, c_int, c_double, dp, dp, ctypes.POINTER(c_long), dp]
    lib.oracle_backend_gn.restype = c_int
    return lib


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a, ctype=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def match_fwd(Xii, Xji, Dii, Dji, Qii=None, Qji=None, p_init=None, *, K=10, lambda0=1e-8, r=3, levels=1,
              conf_min=1.5, max_theta=1e-4, max_dist=math.inf, nthreads=0, lib=None):
    """Run the oracle forward.  Arrays are (H, W, 3) / (H, W, D) / (H, W) / (H, W, 2).

    Returns a dict of numpy arrays: p (H, W, 2) float64, idx (H, W) int32,
    valid (H, W) bool, theta (H, W), xhat (H, W, 3), gap (H, W).
    """
    lib = lib or load()
    H, W = np.shape(Xii)[:2]
    D = np.shape(Dii)[2]
    N = H * W
    Xii, Xji = _f64(Xii, (N, 3)), _f64(Xji, (N, 3))
    Dii, Dji = _f64(Dii, (N, D)), _f64(Dji, (N, D))
    if (Qii is None) != (Qji is None):
        raise ValueError("Qii and Qji must both be given or both be None")
    Qii, Qji = _f64(Qii, (N,)), _f64(Qji, (N,))
    p_init = _f64(p_init, (N, 2))
    p = np.empty((N, 2)); theta = np.empty(N); xhat = np.empty((N, 3)); gap = np.empty(N)
    idx = np.empty(N, np.int32); valid = np.empty(N, np.uint8)
    rc = lib.oracle_match_fwd(H, W, D, _ptr(Xii), _ptr(Xji), _ptr(Dii), _ptr(Dji), _ptr(Qii), _ptr(Qji),
                              _ptr(p_init), int(K), float(lambda0), int(r), int(levels), float(conf_min),
                              float(max_theta), float(max_dist), _ptr(p), _ptr(idx, ctypes.c_int32),
                              _ptr(valid, ctypes.c_uint8), _ptr(theta), _ptr(xhat), _ptr(gap), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_match_fwd failed with %d" % rc)
    return dict(p=p.reshape(H, W, 2), idx=idx.reshape(H, W), valid=valid.reshape(H, W).astype(bool),
                theta=theta.reshape(H, W), xhat=xhat.reshape(H, W, 3), gap=gap.reshape(H, W))


def match_bwd(Xii, Xji, p, valid, grad_p=None, grad_xhat=None, lib=None):
    """Implicit adjoint: returns (dL/dXii, dL/dXji), each (H, W, 3) float64."""
    lib = lib or load()
    H, W = np.shape(Xii)[:2]
    N = H * W
    Xii, Xji = _f64(Xii, (N, 3)), _f64(Xji, (N, 3))
    p = _f64(p, (N, 2))
    valid = np.ascontiguousarray(np.asarray(valid).reshape(N).astype(np.uint8))
    grad_p = _f64(grad_p, (N, 2))
    grad_xhat = _f64(grad_xhat, (N, 3))
    dXii = np.empty((N, 3)); dXji = np.empty((N, 3))
    rc = lib.oracle_match_bwd(H, W, _ptr(Xii), _ptr(Xji), _ptr(p), _ptr(valid, ctypes.c_uint8),
                              _ptr(grad_p), _ptr(grad_xhat), _ptr(dXii), _ptr(dXji))
    if rc != 0:
        raise ValueError("oracle_match_bwd failed with %d" % rc)
    return dXii.reshape(H, W, 3), dXji.reshape(H, W, 3)


def cost_grid(Xii, x, px, py, lib=None):
    """Ray error c(p) of one target point x at the pixels (px, py) (same shape)."""
    lib = lib or load()
    H, W = np.shape(Xii)[:2]
    Xii = _f64(Xii, (H * W, 3))
    x = _f64(x, (3,))
    shape = np.shape(px)
    px = _f64(px).reshape(-1)
    py = _f64(py).reshape(-1)
    out = np.empty(px.size)
    rc = lib.oracle_cost_grid(H, W, _ptr(Xii), _ptr(x), px.size, _ptr(px), _ptr(py), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_cost_grid failed")
    return out.reshape(shape)


def ray_images(Xii, lib=None):
    """(R, Gx, Gy), each (H, W, 3): the ray image and its central-difference gradients."""
    lib = lib or load()
    H, W = np.shape(Xii)[:2]
    X = _f64(Xii, (H * W, 3))
    R, Gx, Gy = (np.empty((H * W, 3)) for _ in range(3))
    if lib.oracle_ray_images(H, W, _ptr(X), _ptr(R), _ptr(Gx), _ptr(Gy)) != 0:
        raise ValueError("oracle_ray_images failed")
    return R.reshape(H, W, 3), Gx.reshape(H, W, 3), Gy.reshape(H, W, 3)


def match_stats(idx, valid):
    """Keyframe statistics of one match set (Sec. 3.4): the number of valid
    matches and the number of distinct reference pixels they land on."""
    idx = np.asarray(idx).reshape(-1)
    valid = np.asarray(valid).reshape(-1).astype(bool)
    return int(valid.sum()), int(np.unique(idx[valid]).size)


# Tracking pose solve defaults (Sec. 3.3; the paper gives no values): confidence
# gate 1.5, ray sigma 0.003, distance sigma 0.1, Huber width 1.345, 10 iterations.
TRACK_DEFAULTS = dict(q_min=1.5, sigma_ray=0.003, sigma_dist=0.1, huber=1.345, iters=10)


def sim3_exp(tau, lib=None):
    """Exp of sim(3), tau = (v, omega, sigma) -> 3x4 [sR | t] (Eq. 1)."""
    lib = lib or load()
    t = _f64(tau, (7,))
    T = np.empty(12)
    lib.oracle_sim3_exp(_ptr(t), _ptr(T))
    return T.reshape(3, 4)


def track_residual(T, Xf_m, Xk_n, lib=None):
    """Ray (3) and distance (1) residuals of one match and their 4x7 Jacobian."""
    lib = lib or load()
    r = np.empty(4); J = np.empty(28)
    lib.oracle_track_residual(_ptr(_f64(T, (12,))), _ptr(_f64(Xf_m, (3,))), _ptr(_f64(Xk_n, (3,))), _ptr(r), _ptr(J))
    return r, J.reshape(4, 7)


def track_pose(Xk, Xf, idx, valid, Qf, Qk, T0, *, q_min=1.5, sigma_ray=0.003, sigma_dist=0.1, huber=1.345,
               iters=10, lib=None):
    """Gauss-Newton IRLS tracking pose (Sec. 3.3).  Returns (T 3x4, info dict)."""
    lib = lib or load()
    H, W = np.shape(Xk)[:2]
    N = H * W
    T = _f64(T0, (12,)).copy()
    cost = ctypes.c_double(); count = ctypes.c_long()
    Hm = np.empty(49); g = np.empty(7)
    idx = np.ascontiguousarray(np.asarray(idx).reshape(N), dtype=np.int32)
    valid = np.ascontiguousarray(np.asarray(valid).reshape(N).astype(np.uint8))
    solved = lib.oracle_track_pose(H, W, _ptr(_f64(Xk, (N, 3))), _ptr(_f64(Xf, (N, 3))), _ptr(idx, ctypes.c_int32),
                                   _ptr(valid, ctypes.c_uint8), _ptr(_f64(Qf, (N,))), _ptr(_f64(Qk, (N,))),
                                   float(q_min), float(sigma_ray), float(sigma_dist), float(huber), int(iters),
                                   _ptr(T), ctypes.byref(cost), ctypes.byref(count), _ptr(Hm), _ptr(g))
    return T.reshape(3, 4), dict(solved=solved, cost=cost.value, count=count.value, H=Hm.reshape(7, 7), g=g)


def fuse(T, Xc, Cc, X, C, lib=None):
    """Canonical pointmap update (Sec. 3.3, Eq. 8): returns the new (Xc, Cc) as fp64 arrays."""
    lib = lib or load()
    shape = np.shape(Xc)
    N = int(np.prod(shape[:-1]))
    Xc2 = _f64(Xc, (N, 3)).copy()
    Cc2 = _f64(Cc, (N,)).copy()
    lib.oracle_fuse(N, _ptr(_f64(T, (12,))), _ptr(Xc2), _ptr(Cc2), _ptr(_f64(X, (N, 3))), _ptr(_f64(C, (N,))))
    return Xc2.reshape(shape), Cc2.reshape(shape[:-1])


def backend_residual(Ti, Tj, Xj_n, Xi_m, lib=None):
    """Ray (3) and distance (1) residuals of one backend match and their 4x7 Jacobians
    w.r.t. the world poses of keyframes i and j (Sec. 3.5, Supp. A)."""
    lib = lib or load()
    r = np.empty(4); Ji = np.empty(28); Jj = np.empty(28)
    ok = lib.oracle_backend_residual(_ptr(_f64(Ti, (12,))), _ptr(_f64(Tj, (12,))), _ptr(_f64(Xj_n, (3,))),
                                     _ptr(_f64(Xi_m, (3,))), _ptr(r), _ptr(Ji), _ptr(Jj))
    if not ok:
        raise ValueError("degenerate point")
    return r, Ji.reshape(4, 7), Jj.reshape(4, 7)


BACKEND_DEFAULTS = dict(q_min=1.5, sigma_ray=0.003, sigma_dist=0.1, huber=1.345, iters=10, step_tol=0.0)


def backend_gn(Xc, Q, edges, idx, valid, T_WC, *, q_min=1.5, sigma_ray=0.003, sigma_dist=0.1, huber=1.345,
               iters=10, step_tol=0.0, lib=None):
    """Backend Gauss-Newton over keyframe poses (Sec. 3.5).  Xc (N, H, W, 3), Q (N, H, W),
    edges (E, 2) as (i, j), idx/valid (E, H, W), T_WC (N, 3, 4).  Returns (T_WC, info)."""
    lib = lib or load()
    N, H, W = np.shape(Xc)[:3]
    E = len(edges)
    HW = H * W
    edges = np.asarray(edges, np.int32).reshape(E, 2)
    ei = np.ascontiguousarray(edges[:, 0]); ej = np.ascontiguousarray(edges[:, 1])
    idx = np.ascontiguousarray(np.asarray(idx).reshape(E * HW), dtype=np.int32)
    valid = np.ascontiguousarray(np.asarray(valid).reshape(E * HW).astype(np.uint8))
    T = _f64(T_WC, (N * 12,)).copy()
    cost = ctypes.c_double(); count = ctypes.c_long(); last = ctypes.c_double()
    applied = lib.oracle_backend_gn(N, H, W, _ptr(_f64(Xc, (N * HW, 3))), _ptr(_f64(Q, (N * HW,))), E,
                                    _ptr(ei, ctypes.c_int32), _ptr(ej, ctypes.c_int32), _ptr(idx, ctypes.c_int32),
                                    _ptr(valid, ctypes.c_uint8), float(q_min), float(sigma_ray), float(sigma_dist),
                                    float(huber), int(iters), float(step_tol), _ptr(T), ctypes.byref(cost),
                                    ctypes.byref(count), ctypes.byref(last))
    return T.reshape(N, 3, 4), dict(applied=applied, cost=cost.value, count=count.value, last_step=last.value)


def max_threads(lib=None) -> int:
    return int((lib or load()).oracle_max_threads())


def match_pair(pair, **kw):
    """Oracle forward on a ``synth.Pair`` with the pair's K and r."""
    args = dict(DEFAULTS, K=pair.K, r=pair.r)
    args.update(kw)
    return match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji, **args)
