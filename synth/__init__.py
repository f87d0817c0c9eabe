"""Seeded synthetic workloads for projective pointmap matching.

The matching method (MASt3R-SLAM, Sec. 3.2) consumes two pointmaps X^i_i, X^j_i
(H x W x 3, both expressed in camera i), two descriptor maps D^i_i, D^j_i
(H x W x d) and optional per-pixel descriptor confidences Q^i_i, Q^j_i
(Sec. 3.1).  The paper's inputs come from the MASt3R network on TUM / 7-Scenes /
EuRoC frames at max side 512 (Sec. 4); neither the network nor the datasets are
available here, so this module builds stand-ins of the same shape:

* X^i_i: a smooth procedural surface seen by a pinhole camera with focal
  f = max(W, H) / 2 and centre ((W-1)/2, (H-1)/2), depth
  z = 2 + 0.3 sin(3u) cos(2v) + 0.1 u + 0.05 v.
* X^j_i: the same surface sampled on a grid shifted by a per-edge offset in
  U(-2, 2)^2 px, moved by a random Sim(3) (rotation <= 10 deg about a uniform
  axis, |t| <= 0.1, scale in [0.9, 1.1]) and perturbed by N(0, 1e-3^2) noise.
* D: unit-norm 24-dim descriptors from a smooth random field (8 sinusoids per
  channel, about 8 cycles across the long side) plus N(0, 0.05^2) noise; the
  query descriptor is the field evaluated at the pinhole projection of the
  query point, so the true correspondence is where the field agrees.
* Q: uniform in [1, 5].

This module holds no arithmetic of the matching method itself (no ray
normalisation, no Levenberg-Marquardt, no refine); it only draws inputs.  All
draws use numpy's PCG64 generator with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

DESC_DIM = 24


@dataclass
class Pair:
    """One matching problem: frame i (reference) and the query pointmap X^j_i."""

    H: int
    W: int
    Xii: np.ndarray            # (H, W, 3) float32
    Xji: np.ndarray            # (H, W, 3) float32
    Dii: np.ndarray            # (H, W, D) float32
    Dji: np.ndarray            # (H, W, D) float32
    Qii: np.ndarray | None     # (H, W) float32
    Qji: np.ndarray | None     # (H, W) float32
    K: int = 10                # LM iterations
    r: int = 3                 # refine radius
    # Ground truth of the generator (not an input of the method): the pinhole
    # projection of every query point into camera i, (H, W, 2) as (x, y).
    proj: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def D(self) -> int:
        return self.Dii.shape[2]

    @property
    def N(self) -> int:
        return self.H * self.W


def camera(H: int, W: int):
    f = max(W, H) / 2.0
    return f, (W - 1) / 2.0, (H - 1) / 2.0


def _depth(u, v):
    return 2.0 + 0.3 * np.sin(3.0 * u) * np.cos(2.0 * v) + (0.1 * u + 0.05 * v)


def surface_points(H: int, W: int, xs, ys) -> np.ndarray:
    """Surface point seen through pixel (xs, ys) of the pinhole camera (float64)."""
    f, cx, cy = camera(H, W)
    u = (np.asarray(xs, np.float64) - cx) / f
    v = (np.asarray(ys, np.float64) - cy) / f
    z = _depth(u, v)
    return np.stack([z * u, z * v, z], axis=-1)


def pixel_grid(H: int, W: int):
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    return xs, ys


def pinhole_project(H: int, W: int, P: np.ndarray) -> np.ndarray:
    """Pixel (x, y) of points P (..., 3) under the generator's pinhole camera."""
    f, cx, cy = camera(H, W)
    return np.stack([f * P[..., 0] / P[..., 2] + cx, f * P[..., 1] / P[..., 2] + cy], axis=-1)


def random_rotation(rng: np.random.Generator, max_deg: float) -> np.ndarray:
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = math.radians(rng.uniform(0.0, max_deg))
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * k + (1.0 - math.cos(ang)) * (k @ k)


def random_sim3(rng: np.random.Generator, max_deg=10.0, max_t=0.1, smin=0.9, smax=1.1):
    R = random_rotation(rng, max_deg)
    tdir = rng.normal(size=3)
    tdir /= np.linalg.norm(tdir)
    t = tdir * rng.uniform(0.0, max_t)
    s = rng.uniform(smin, smax)
    return s, R, t


class DescriptorField:
    """Smooth random field F: R^2 -> R^D, F_d(x) = sum_k a_dk sin(w_dk . x + phi_dk)."""

    def __init__(self, rng: np.random.Generator, H: int, W: int, D: int = DESC_DIM,
                 n_waves: int = 8, cycles: float = 8.0):
        sig = 2.0 * math.pi * cycles / max(W, H)
        self.omega = rng.normal(0.0, sig, size=(D, n_waves, 2))
        self.amp = rng.normal(0.0, 1.0, size=(D, n_waves))
        self.phase = rng.uniform(0.0, 2.0 * math.pi, size=(D, n_waves))

    def __call__(self, xs, ys, chunk: int = 16384) -> np.ndarray:
        # float64 on torch's multi-threaded CPU kernels, in chunks of points;
        # numpy's float64 sin is ~8x slower and this runs for every edge.
        import torch
        xs = np.asarray(xs, np.float64)
        ys = np.asarray(ys, np.float64)
        shape = xs.shape
        xf = torch.from_numpy(np.ascontiguousarray(xs.reshape(-1)))
        yf = torch.from_numpy(np.ascontiguousarray(ys.reshape(-1)))
        wx = torch.from_numpy(self.omega[..., 0])
        wy = torch.from_numpy(self.omega[..., 1])
        ph = torch.from_numpy(self.phase)
        am = torch.from_numpy(self.amp)
        out = torch.empty((xf.numel(), self.amp.shape[0]), dtype=torch.float64)
        for s in range(0, xf.numel(), chunk):
            x = xf[s:s + chunk, None, None]
            y = yf[s:s + chunk, None, None]
            out[s:s + chunk] = (am * torch.sin(wx * x + wy * y + ph)).sum(-1)
        return out.numpy().reshape(*shape, -1)


def _unit_rows(a: np.ndarray) -> np.ndarray:
    return a / np.linalg.norm(a, axis=-1, keepdims=True)


def make_pair(H: int, W: int, seed: int, *, K: int = 10, r: int = 3, conf: bool = True,
              D: int = DESC_DIM, max_deg: float = 10.0, max_t: float = 0.1,
              scale_range=(0.9, 1.1), shift_px: float = 2.0, noise: float = 1e-3,
              desc_noise: float = 0.05, cycles: float = 8.0) -> Pair:
    """The synthetic pair described in the module docstring."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs, ys = pixel_grid(H, W)
    Xii = surface_points(H, W, xs, ys)

    d = rng.uniform(-shift_px, shift_px, size=2)
    P = surface_points(H, W, xs + d[0], ys + d[1])
    s, R, t = random_sim3(rng, max_deg, max_t, *scale_range)
    Xji = s * (P @ R.T) + t
    Xji = Xji + rng.normal(0.0, noise, size=Xji.shape)
    # Ground truth from the float32 points the matcher will actually see.
    proj = pinhole_project(H, W, Xji.astype(np.float32).astype(np.float64))

    field_ = DescriptorField(rng, H, W, D, cycles=cycles)
    Dii = _unit_rows(field_(xs, ys) + rng.normal(0.0, desc_noise, size=(H, W, D)))
    Dji = _unit_rows(field_(proj[..., 0], proj[..., 1]) + rng.normal(0.0, desc_noise, size=(H, W, D)))
    if conf:
        Qii = rng.uniform(1.0, 5.0, size=(H, W))
        Qji = rng.uniform(1.0, 5.0, size=(H, W))
    else:
        Qii = Qji = None
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    return Pair(H, W, f32(Xii), f32(Xji), f32(Dii), f32(Dji), f32(Qii), f32(Qji), K=K, r=r,
                proj=proj, meta=dict(seed=seed, shift=d.tolist(), scale=s, t=t.tolist(), R=R.tolist()))


def identity_pair(H: int, W: int, seed: int, D: int = DESC_DIM) -> Pair:
    """X^j_i = X^i_i and D^j_i = D^i_i: every pixel must match itself."""
    p = make_pair(H, W, seed, D=D, conf=False)
    return Pair(H, W, p.Xii.copy(), p.Xii.copy(), p.Dii.copy(), p.Dii.copy(), None, None,
                proj=np.stack(pixel_grid(H, W), -1), meta=dict(seed=seed, identity=True))


def distorted_camera_rays(H: int, W: int, xs, ys, k1: float = -0.2, k2: float = 0.05) -> np.ndarray:
    """Un-normalised ray directions of a radially distorted central camera.

    The ray through pixel (x, y) points along (u d(r), v d(r), 1) with
    u = (x - cx) / f, v = (y - cy) / f, r^2 = u^2 + v^2, d(r) = 1 + k1 r^2 + k2 r^4.
    """
    f, cx, cy = camera(H, W)
    u = (np.asarray(xs, np.float64) - cx) / f
    v = (np.asarray(ys, np.float64) - cy) / f
    r2 = u * u + v * v
    dist = 1.0 + k1 * r2 + k2 * r2 * r2
    return np.stack([u * dist, v * dist, np.ones_like(u)], -1)


def distorted_camera_pointmap(H: int, W: int, seed: int, k1: float = -0.2, k2: float = 0.05,
                              depth_jitter: float = 0.5) -> np.ndarray:
    """A generic central camera: radially distorted rays with random depths along them."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs, ys = pixel_grid(H, W)
    dirs = distorted_camera_rays(H, W, xs, ys, k1, k2)
    depth = 1.0 + depth_jitter * rng.uniform(size=(H, W, 1))
    return np.ascontiguousarray(dirs * depth, dtype=np.float32)


def config_pair(config: int, edge: int = 0) -> Pair:
    """The single-pair workloads: 1 = 64x48 without confidences, 2 = 512x384 with."""
    seed = 1000 * config + edge
    if config == 1:
        return make_pair(48, 64, seed, K=10, r=3, conf=False)
    if config == 2:
        return make_pair(384, 512, seed, K=10, r=3, conf=True)
    if config == 5:
        return make_pair(384, 512, seed, K=10, r=3, conf=True)
    raise ValueError(config)


def batched_uniform(n_edges: int = 64, H: int = 384, W: int = 512, seed_base: int = 3000):
    """64 independent 512x384 edges, K = 10, r = 3 (one Sim(3) per edge)."""
    return [make_pair(H, W, seed_base + e, K=10, r=3, conf=True) for e in range(n_edges)]


def batched_uneven_spec(seed_base: int = 4000):
    """Shapes, iteration counts and radii of the mixed-resolution batch.

    40 edges at 512x384, 32 at 384x512 and 24 at 512x288 (W x H), with
    K ~ U{5..15} and r ~ U{2, 3, 4} per edge, drawn from one seeded stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed_base))
    dims = [(384, 512)] * 40 + [(512, 384)] * 32 + [(288, 512)] * 24   # (H, W)
    Ks = rng.integers(5, 16, size=len(dims))
    rs = rng.integers(2, 5, size=len(dims))
    return [(H, W, int(K), int(r)) for (H, W), K, r in zip(dims, Ks, rs)]


def batched_uneven(seed_base: int = 4000, limit: int | None = None):
    spec = batched_uneven_spec(seed_base)
    if limit is not None:
        spec = spec[:limit]
    return [make_pair(H, W, seed_base + 1 + e, K=K, r=r, conf=True) for e, (H, W, K, r) in enumerate(spec)]


@dataclass
class TrackingProblem:
    """Inputs of the tracking pose solve (Sec. 3.3) with its ground truth.

    Xk: canonical keyframe points (measured), Xf: current-frame points,
    idx[n]: frame pixel matched to keyframe pixel n, valid, Qf, Qk confidences,
    T_true: the 3x4 Sim(3) [sR | t] with Xk[n] = T_true Xf[idx[n]] (+ noise)
    for inliers; `outlier` marks the matches displaced on purpose.
    """

    H: int
    W: int
    Xk: np.ndarray
    Xf: np.ndarray
    idx: np.ndarray
    valid: np.ndarray
    Qf: np.ndarray
    Qk: np.ndarray
    T_true: np.ndarray
    outlier: np.ndarray


def make_tracking(H: int, W: int, seed: int, *, max_deg: float = 5.0, max_t: float = 0.05,
                  scale_range=(0.95, 1.05), noise: float = 0.0, outlier_frac: float = 0.0,
                  outlier_mag: float = 0.5, valid_frac: float = 0.95, pure_rotation: bool = False) -> TrackingProblem:
    """Frame points on the procedural pinhole surface, a random Sim(3), matches
    that shift pixels by a few columns, optional noise and gross outliers."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs, ys = pixel_grid(H, W)
    Xf = surface_points(H, W, xs, ys)
    if pure_rotation:
        s, R, t = 1.0, random_rotation(rng, max_deg), np.zeros(3)
    else:
        s, R, t = random_sim3(rng, max_deg, max_t, *scale_range)
    T = np.concatenate([s * R, t[:, None]], 1)
    shift = rng.integers(-3, 4)
    mx = np.clip(xs.astype(int) + shift, 0, W - 1)
    idx = (ys.astype(int) * W + mx).reshape(-1)
    P = Xf.reshape(-1, 3)[idx]
    Xk = P @ T[:, :3].T + T[:, 3]
    Xk = Xk + rng.normal(0.0, noise, size=Xk.shape) if noise > 0 else Xk
    outlier = rng.uniform(size=H * W) < outlier_frac
    Xk[outlier] += rng.normal(0.0, outlier_mag, size=(int(outlier.sum()), 3))
    valid = rng.uniform(size=H * W) < valid_frac
    Qf = rng.uniform(1.0, 5.0, size=H * W)
    Qk = rng.uniform(1.0, 5.0, size=H * W)
    f32 = lambda a, shape: np.ascontiguousarray(a.reshape(shape), dtype=np.float32)
    return TrackingProblem(H, W, f32(Xk, (H, W, 3)), f32(Xf, (H, W, 3)), idx.reshape(H, W).astype(np.int32),
                           valid.reshape(H, W), f32(Qf, (H, W)), f32(Qk, (H, W)), T, outlier.reshape(H, W))


@dataclass
class FusionProblem:
    """Inputs of the canonical pointmap update (Sec. 3.3, Eq. 8).

    Xc, Cc: the keyframe's canonical pointmap and its summed confidence;
    X: a frame's prediction of the keyframe pixels' points in the frame's
    coordinates (X^k_f), C its confidence; T: the 3x4 Sim(3) T_kf with
    T X = P (+ noise) for the keyframe-frame points P.
    """

    H: int
    W: int
    Xc: np.ndarray
    Cc: np.ndarray
    X: np.ndarray
    C: np.ndarray
    T: np.ndarray
    P: np.ndarray


def make_fusion(H: int, W: int, seed: int, *, noise: float = 1e-2, zero_conf_frac: float = 0.02,
                max_deg: float = 10.0, max_t: float = 0.1) -> FusionProblem:
    """Keyframe surface points P; canonical map = P + noise with confidence
    U(0.5, 20) (a few zeros); the frame's view of P through the inverse of a
    random Sim(3) with its own noise and confidence U(1, 5) (a few zeros)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs, ys = pixel_grid(H, W)
    P = surface_points(H, W, xs, ys).reshape(-1, 3)
    s, R, t = random_sim3(rng, max_deg, max_t)
    T = np.concatenate([s * R, t[:, None]], 1)
    Xc = P + rng.normal(0.0, noise, size=P.shape)
    Cc = rng.uniform(0.5, 20.0, size=H * W)
    Cc[rng.uniform(size=H * W) < zero_conf_frac] = 0.0
    Pn = P + rng.normal(0.0, noise, size=P.shape)
    X = ((Pn - t) @ R) / s                      # T^-1 applied to the noisy points
    C = rng.uniform(1.0, 5.0, size=H * W)
    C[rng.uniform(size=H * W) < zero_conf_frac] = 0.0
    both = rng.uniform(size=H * W) < zero_conf_frac
    Cc[both] = 0.0
    C[both] = 0.0
    f32 = lambda a, shape: np.ascontiguousarray(a.reshape(shape), dtype=np.float32)
    return FusionProblem(H, W, f32(Xc, (H, W, 3)), f32(Cc, (H, W)), f32(X, (H, W, 3)), f32(C, (H, W)), T,
                         P.reshape(H, W, 3))


@dataclass
class BackendProblem:
    """Inputs of the backend pose-graph optimisation (Sec. 3.5).

    N keyframes of one H x W resolution.  Xc[k]: canonical pointmap of keyframe
    k in its own camera; Q[k]: its confidence; edges[e] = (i, j) with idx[e][n]
    the pixel of keyframe i matched to pixel n of keyframe j and valid[e][n];
    T_true[k] / T_init[k]: 3x4 world poses (keyframe 0 is the same in both).
    """

    N: int
    H: int
    W: int
    Xc: np.ndarray
    Q: np.ndarray
    edges: np.ndarray
    idx: np.ndarray
    valid: np.ndarray
    T_true: np.ndarray
    T_init: np.ndarray


def _sim3_matrix(s, R, t):
    return np.concatenate([s * R, np.asarray(t, np.float64)[:, None]], 1)


def _sim3_mul(A, B):
    return np.concatenate([A[:, :3] @ B[:, :3], (A[:, :3] @ B[:, 3] + A[:, 3])[:, None]], 1)


def _sim3_inv(T):
    s = np.cbrt(np.linalg.det(T[:, :3]))
    Ri = T[:, :3].T / (s * s)
    return np.concatenate([Ri, (-Ri @ T[:, 3])[:, None]], 1)


def make_backend(N: int, H: int, W: int, seed: int, *, loops: int = 1, scramble: bool = True,
                 noise: float = 0.0, outlier_frac: float = 0.0, valid_frac: float = 0.95,
                 init_deg: float = 2.0, init_t: float = 0.02, init_scale=(0.98, 1.02)) -> BackendProblem:
    """World points on the procedural surface seen by N keyframes along a path.

    Keyframe k's pixel pi_k(p) sees world point P[p] (pi_k a random pixel
    permutation when `scramble`, else the identity), so an edge (i, j) matches
    pixel n of j to pi_i(pi_j^-1(n)).  Edges: both directions between
    consecutive keyframes, plus `loops` closures (k, N-1-k).  Initial poses:
    the true ones times a small random Sim(3), keyframe 0 exact."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs, ys = pixel_grid(H, W)
    P0 = surface_points(H, W, xs, ys).reshape(-1, 3)
    HW = H * W
    T_true = np.zeros((N, 3, 4))
    T_init = np.zeros((N, 3, 4))
    for k in range(N):
        if k == 0:
            T_true[k] = _sim3_matrix(1.0, np.eye(3), np.zeros(3))
        else:
            s, R, t = random_sim3(rng, 8.0, 0.15, 0.9, 1.1)
            T_true[k] = _sim3_mul(T_true[k - 1], _sim3_matrix(s, R, t))
        ds, dR, dt = random_sim3(rng, init_deg, init_t, *init_scale)
        T_init[k] = T_true[k] if k == 0 else _sim3_mul(_sim3_matrix(ds, dR, dt), T_true[k])
    perms = [rng.permutation(HW) if scramble else np.arange(HW) for _ in range(N)]
    Xc = np.zeros((N, HW, 3))
    for k in range(N):
        Tinv = _sim3_inv(T_true[k])
        Xk = np.zeros((HW, 3))
        Xk[perms[k]] = P0 @ Tinv[:, :3].T + Tinv[:, 3]
        if noise > 0:
            Xk = Xk + rng.normal(0.0, noise, size=Xk.shape)
        Xc[k] = Xk
    pairs = []
    for k in range(1, N):
        pairs += [(k - 1, k), (k, k - 1)]
    for c in range(loops):
        i, j = c, N - 1 - c
        if j - i > 1:
            pairs.append((i, j))
    E = len(pairs)
    idx = np.zeros((E, HW), np.int32)
    valid = np.zeros((E, HW), bool)
    inv_perm = [np.argsort(p) for p in perms]
    for e, (i, j) in enumerate(pairs):
        idx[e] = perms[i][inv_perm[j]]
        valid[e] = rng.uniform(size=HW) < valid_frac
        bad = rng.uniform(size=HW) < outlier_frac
        idx[e][bad] = rng.integers(0, HW, size=int(bad.sum()))
    Q = rng.uniform(1.0, 5.0, size=(N, HW))
    f32 = lambda a, shape: np.ascontiguousarray(a.reshape(shape), dtype=np.float32)
    return BackendProblem(N, H, W, f32(Xc, (N, H, W, 3)), f32(Q, (N, H, W)), np.array(pairs, np.int32),
                          idx.reshape(E, H, W), valid.reshape(E, H, W), T_true, T_init)
