"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes a loaded oracle library (``oracle.load(path)``)
and raises AssertionError when the oracle disagrees with:

* closed forms: the pinhole projection a pinhole ray image must reproduce,
  the angle to the nearest border ray, the analytic derivative of pinhole
  rays, the pinhole projection Jacobian (Supp. A, projection Jacobian);
* special cases: identity pairs, planted descriptors, exact-threshold gates;
* invariants: depth independence of rays for a central camera (Sec. 3.1),
  orthogonality of the backward to the radial direction (Supp. A, Eq. norm_jac);
* brute force: exhaustive scans of the ray error on tiny generic cameras;
* the paper's convergence statement (Sec. 3.2: ten LM iterations suffice for
  nearly every valid pixel);
* finite differences of the loss through the forward, and autograd through an
  independent unrolled statement of the solver.

``test_oracle_pins.py`` runs them on the oracle; ``test_oracle_mutants.py``
runs them on deliberately broken copies of the oracle to show each plausible
mistake is caught.
"""
from __future__ import annotations

import functools
import math

import numpy as np

import oracle
import synth


def fwd(lib, Xii, Xji, Dii=None, Dji=None, Qii=None, Qji=None, p_init=None, **kw):
    H, W = Xii.shape[:2]
    if Dii is None:
        Dii = np.ones((H, W, 1))
        Dji = np.ones((H, W, 1))
    args = dict(oracle.DEFAULTS)
    args.update(kw)
    args.setdefault("nthreads", 1)
    return oracle.match_fwd(Xii, Xji, Dii, Dji, Qii, Qji, p_init, lib=lib, **args)


def pinhole_rays(H, W, f=None):
    f0, cx, cy = synth.camera(H, W)
    f = f0 if f is None else f
    xs, ys = synth.pixel_grid(H, W)
    return np.stack([(xs - cx) / f, (ys - cy) / f, np.ones_like(xs)], -1), f, cx, cy


@functools.lru_cache(maxsize=None)
def _pair(H, W, seed, conf=True):
    return synth.make_pair(H, W, seed, conf=conf)


# ---------------------------------------------------------------- forward pins

def pin_identity(lib):
    """X^j_i = X^i_i, D^j_i = D^i_i: every pixel returns to itself (identity init)."""
    for (H, W) in [(48, 64), (7, 13)]:
        p = synth.identity_pair(H, W, seed=11)
        o = fwd(lib, p.Xii, p.Xji, p.Dii, p.Dji)
        xs, ys = synth.pixel_grid(H, W)
        assert np.abs(o["p"][..., 0] - xs).max() <= 1e-12, "identity: p_x"
        assert np.abs(o["p"][..., 1] - ys).max() <= 1e-12, "identity: p_y"
        assert o["theta"].max() <= 1e-7, "identity: theta"
        assert (o["idx"] == np.arange(H * W).reshape(H, W)).all(), "identity: idx"
        assert o["valid"].all(), "identity: valid"
        # xhat is X^i_i sampled at p* = the pixel itself.
        assert np.abs(o["xhat"] - p.Xii).max() <= 1e-12, "identity: xhat"


def _interior_true_match(pair, margin):
    pr = pair.proj
    return ((pr[..., 0] >= margin) & (pr[..., 0] <= pair.W - 1 - margin)
            & (pr[..., 1] >= margin) & (pr[..., 1] <= pair.H - 1 - margin))


def pin_pinhole(lib):
    """A pinhole ray image: the converged match is the pinhole projection of the query.

    The oracle differs from the projection only by the bilinear interpolation
    of the ray image, which shrinks with resolution (1e-2 px at 64x48 and
    2e-3 px at 160x120 bound it); queries whose projection is within 1 px of
    the border are left out because they can converge onto the clamped edge.
    """
    for (H, W, tol, seed) in [(48, 64, 1e-2, 1001), (120, 160, 2e-3, 77)]:
        pair = _pair(H, W, seed, False)
        o = fwd(lib, pair.Xii, pair.Xji)
        m = _interior_true_match(pair, 1.0)
        assert m.mean() > 0.5
        err = np.abs(o["p"] - pair.proj)[m]
        assert err.max() <= tol, "pinhole: max |p* - pi(x)| = %g" % err.max()
        assert o["valid"][m].all(), "pinhole: interior matches must be valid"
        assert o["theta"][m].max() <= 1e-12, "pinhole: zero residual"


def pin_brute_force(lib):
    """Tiny generic central cameras with radial distortion: for queries inside the
    field of view, LM reaches the global minimiser of the ray error found by an
    exhaustive scan (1/8 px, then 1/128 px around the best cell).  Queries whose
    rays lie outside the field of view have no zero-residual match and must be
    invalid."""
    for (H, W, seed) in [(9, 12, 5), (12, 16, 6)]:
        Xii = synth.distorted_camera_pointmap(H, W, seed)
        rng = np.random.Generator(np.random.PCG64(seed))
        n_in, n_out = 14, 4
        # In-FOV query rays: the camera's rays through random fractional pixels.
        fx = rng.uniform(0.5, W - 1.5, n_in)
        fy = rng.uniform(0.5, H - 1.5, n_in)
        rays_in = synth.distorted_camera_rays(H, W, fx, fy)
        # Out-of-FOV rays: beyond a random border by 1.5 - 3 px.
        side = rng.integers(0, 4, n_out)
        ox = np.where(side == 0, -rng.uniform(1.5, 3, n_out), np.where(side == 1, W - 1 + rng.uniform(1.5, 3, n_out), rng.uniform(0, W - 1, n_out)))
        oy = np.where(side == 2, -rng.uniform(1.5, 3, n_out), np.where(side == 3, H - 1 + rng.uniform(1.5, 3, n_out), rng.uniform(0, H - 1, n_out)))
        rays_out = synth.distorted_camera_rays(H, W, ox, oy)
        pts = np.concatenate([rays_in, rays_out]) * rng.uniform(0.5, 3.0, n_in + n_out)[:, None]
        n_q = n_in + n_out
        flat = rng.choice(H * W, size=n_q, replace=False)
        qy, qx = flat // W, flat % W
        Xji = np.tile(np.array([0.0, 0.0, 1.0]), (H, W, 1))
        Xji[qy, qx] = pts
        o = fwd(lib, Xii, Xji)
        gx = np.arange(0, (W - 1) * 8 + 1) / 8.0
        gy = np.arange(0, (H - 1) * 8 + 1) / 8.0
        GX, GY = np.meshgrid(gx, gy)
        for k in range(n_q):
            lm_p = o["p"][qy[k], qx[k]]
            if k >= n_in:
                assert not o["valid"][qy[k], qx[k]], "brute force: out-of-FOV query must be invalid"
                continue
            c = oracle.cost_grid(Xii, pts[k], GX, GY, lib=lib)
            j = np.unravel_index(np.argmin(c), c.shape)
            bx, by = GX[j], GY[j]
            fxs = np.clip(bx + np.arange(-32, 33) / 128.0, 0, W - 1)
            fys = np.clip(by + np.arange(-32, 33) / 128.0, 0, H - 1)
            FX, FY = np.meshgrid(fxs, fys)
            cf = oracle.cost_grid(Xii, pts[k], FX, FY, lib=lib)
            jf = np.unravel_index(np.argmin(cf), cf.shape)
            best = cf[jf]
            lm_c = oracle.cost_grid(Xii, pts[k], lm_p[:1], lm_p[1:], lib=lib)[0]
            assert lm_c <= best + 1e-12, "brute force: LM cost %g above scan %g" % (lm_c, best)
            assert np.abs(lm_p - [FX[jf], FY[jf]]).max() <= 2.0 / 128, "brute force: location"
            assert o["valid"][qy[k], qx[k]], "brute force: in-FOV query must be valid"


def pin_depth_invariance(lib):
    """Rays do not depend on depth (Sec. 3.1): scaling any point by 2^k changes nothing."""
    pair = _pair(48, 64, 1001)
    rng = np.random.Generator(np.random.PCG64(3))
    si = 2.0 ** rng.integers(-3, 4, size=(pair.H, pair.W, 1))
    sj = 2.0 ** rng.integers(-3, 4, size=(pair.H, pair.W, 1))
    a = fwd(lib, pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji)
    b = fwd(lib, pair.Xii * si, pair.Xji * sj, pair.Dii, pair.Dji, pair.Qii, pair.Qji)
    for k in ("p", "idx", "valid", "theta"):
        assert np.array_equal(a[k], b[k]), "depth invariance: %s" % k


def pin_border_angle(lib):
    """Queries outside the FOV converge to the nearest border ray; the residual angle
    equals the closed-form angle between the query ray and that border ray (Eq. 3)."""
    for (H, W, axis) in [(31, 40, 0), (40, 31, 1)]:
        R, f, cx, cy = pinhole_rays(H, W)
        Xii = R * 2.0
        angles = [1e-3, 3e-2, 0.3, 0.7]
        Xji = np.tile(np.array([0.0, 0.0, 1.0]), (H, W, 1))
        ub = ((W - 1) - cx) / f if axis == 0 else ((H - 1) - cy) / f
        queries = []
        for k, ang in enumerate(angles):
            uq = math.tan(math.atan(ub) + ang)
            vec = np.array([uq, 0.0, 1.0]) if axis == 0 else np.array([0.0, uq, 1.0])
            qy, qx = 2 + k, 3
            Xji[qy, qx] = vec * 1.7
            queries.append((qy, qx, ang))
        # The method's own 10 iterations: with the coordinate on the border held,
        # the other one converges along the border.
        o = fwd(lib, Xii, Xji, K=10)
        for qy, qx, ang in queries:
            th = o["theta"][qy, qx]
            assert abs(th - ang) <= 1e-9 * max(1.0, ang), "border angle: %g vs %g" % (th, ang)
            # Eq. 3: |psi1 - psi2|^2 = 2 (1 - cos theta) with the border ray.
            pb = o["p"][qy, qx]
            expect_edge = (W - 1) if axis == 0 else (H - 1)
            assert abs(pb[axis] - expect_edge) <= 1e-12, "border angle: match not on the border"


def pin_gradient_images(lib):
    """Central-difference gradient images of a pinhole ray image match the analytic
    derivative of the pinhole ray (Sec. 3.1 rays) up to O(1/f^2) truncation."""
    H, W = 30, 44
    R, f, cx, cy = pinhole_rays(H, W)
    Rn, Gx, Gy = oracle.ray_images(R * 3.0, lib=lib)
    n = np.linalg.norm(R, axis=-1, keepdims=True)
    psi = R / n
    ex = np.array([1.0 / f, 0, 0])
    ey = np.array([0, 1.0 / f, 0])
    ax = (ex - psi * (psi @ ex)[..., None]) / n
    ay = (ey - psi * (psi @ ey)[..., None]) / n
    sl = (slice(1, H - 1), slice(1, W - 1))
    assert np.abs(Rn - psi).max() <= 1e-15, "ray image"
    scale = np.abs(ax[sl]).max()
    assert np.abs(Gx[sl] - ax[sl]).max() <= 2.0 / f ** 2 * scale, "Gx"
    assert np.abs(Gy[sl] - ay[sl]).max() <= 2.0 / f ** 2 * scale, "Gy"
    # One-sided at the border: forward difference of the first two columns/rows.
    assert np.allclose(Gx[:, 0], Rn[:, 1] - Rn[:, 0], rtol=0, atol=1e-15), "Gx border"
    assert np.allclose(Gy[-1], Rn[-1] - Rn[-2], rtol=0, atol=1e-15), "Gy border"


def pin_convergence(lib):
    """Sec. 3.2 (LM convergence): by the tenth iteration nearly every valid pixel
    has converged.  The 10th step moves at most 1e-6 px for >= 99.9 % of valid
    pixels at 512x384."""
    pair = _pair(384, 512, 2000)
    a = fwd(lib, pair.Xii, pair.Xji, K=9, nthreads=0)
    b = fwd(lib, pair.Xii, pair.Xji, K=10, nthreads=0)
    m = b["valid"] & _interior_true_match(pair, 1.0)
    step = np.abs(b["p"] - a["p"]).max(-1)[m]
    assert (step <= 1e-6).mean() >= 0.999, "convergence: %g" % (step <= 1e-6).mean()
    assert m.mean() > 0.5


def pin_refine_planted(lib):
    """Feature refine (Sec. 3.2): a query descriptor planted equal to the descriptor of
    a pixel inside the window selects that pixel, including at the window's corners
    and where the window is clipped by the image border."""
    pair = _pair(48, 64, 1001, False)
    base = fwd(lib, pair.Xii, pair.Xji, pair.Dii, pair.Dji)
    r = 3
    Dji = pair.Dji.astype(np.float64).copy()
    rng = np.random.Generator(np.random.PCG64(9))
    H, W = pair.H, pair.W
    m0 = np.floor(base["p"] + 0.5).astype(int)
    want = {}
    offsets = [(-r, -r), (r, r), (-r, r), (r, -r), (0, 0), (1, -2)]
    ys, xs = np.nonzero(base["valid"])
    pick = rng.choice(len(ys), size=60, replace=False)
    for k, j in enumerate(pick):
        y, x = ys[j], xs[j]
        dx, dy = offsets[k % len(offsets)]
        mx, my = m0[y, x, 0] + dx, m0[y, x, 1] + dy
        if not (0 <= mx < W and 0 <= my < H):
            continue
        Dji[y, x] = pair.Dii[my, mx]
        want[(y, x)] = my * W + mx
    o = fwd(lib, pair.Xii, pair.Xji, pair.Dii, Dji, r=r)
    assert len(want) > 20
    for (y, x), m in want.items():
        assert o["idx"][y, x] == m, "planted refine at (%d,%d): %d vs %d" % (y, x, o["idx"][y, x], m)
    # r = 0: the refined match is p* rounded half up.
    o0 = fwd(lib, pair.Xii, pair.Xji, pair.Dii, pair.Dji, r=0)
    assert (o0["idx"] == m0[..., 1] * W + m0[..., 0]).all(), "r = 0"


def pin_refine_ties(lib):
    """Equal scores: the first maximum in row-major window order wins."""
    pair = _pair(48, 64, 1001, False)
    H, W = pair.H, pair.W
    Dc = np.ones((H, W, 4)) / 2.0
    o = fwd(lib, pair.Xii, pair.Xji, Dc, Dc, r=2)
    m0 = np.floor(o["p"] + 0.5).astype(int)
    fx = np.maximum(m0[..., 0] - 2, 0)
    fy = np.maximum(m0[..., 1] - 2, 0)
    assert (o["idx"] == fy * W + fx).all(), "ties: first in row-major order"
    assert (o["gap"] == 0).all(), "ties: zero gap"


def pin_conf_gate(lib):
    """Match confidence q = sqrt(Q^i_i[m] Q^j_i[n]) (Sec. 3.3) gated at q >= q_min,
    with m the refined match (not the query pixel): exact-threshold cases on a
    warped pair, where m and n differ."""
    pair = _pair(48, 64, 1001, False)
    H, W = pair.H, pair.W
    base = fwd(lib, pair.Xii, pair.Xji, pair.Dii, pair.Dji)
    rng = np.random.Generator(np.random.PCG64(5))
    Qi = rng.choice([0.5, 1.0, 2.0, 4.0], size=(H, W))
    idx = np.where(base["idx"] >= 0, base["idx"], 0)
    assert (idx != np.arange(H * W).reshape(H, W))[base["valid"]].mean() > 0.5
    # Q^j_i chosen so that q is exactly 1.5 (passes) or just below (fails).
    below = rng.uniform(size=(H, W)) < 0.5
    target = np.where(below, 2.25 * (1 - 1e-9), 2.25)
    Qj = target / Qi.reshape(-1)[idx]
    o = fwd(lib, pair.Xii, pair.Xji, pair.Dii, pair.Dji, Qi, Qj, conf_min=1.5)
    assert np.array_equal(o["idx"], base["idx"]), "the gate must not change the match"
    assert np.array_equal(o["valid"], base["valid"] & ~below), "confidence gate"


def pin_dist_gate(lib):
    """3D distance gate (Sec. 3.2): same rays at 1.5x depth match pixel-to-pixel with
    distance 0.5 |X^i_i|; the gate keeps exactly those within max_dist."""
    p = synth.identity_pair(24, 32, seed=4)
    Xj = p.Xii.astype(np.float64) * 1.5
    dist = 0.5 * np.linalg.norm(p.Xii.astype(np.float64), axis=-1)
    thr = float(np.median(dist))
    o = fwd(lib, p.Xii, Xj, p.Dii, p.Dji, max_dist=thr)
    assert np.array_equal(o["valid"], dist <= thr), "distance gate"
    o = fwd(lib, p.Xii, Xj, p.Dii, p.Dji)
    assert o["valid"].all(), "distance gate off by default"


def pin_theta_gate(lib):
    """Residual-angle gate: matches with theta above max_theta are invalid."""
    pair = _pair(48, 64, 1001, False)
    o = fwd(lib, pair.Xii, pair.Xji, max_theta=math.inf)
    o2 = fwd(lib, pair.Xii, pair.Xji, max_theta=1e-4)
    assert o["valid"].all()
    assert np.array_equal(o2["valid"], o["theta"] <= 1e-4)
    outside = ~_interior_true_match(pair, -0.5)
    assert not o2["valid"][outside].any(), "queries beyond the FOV must be invalid"


def pin_bad_inputs(lib):
    """Non-finite or zero query points and non-finite initial pixels give invalid
    matches; bad reference pixels do not poison matches elsewhere."""
    pair = _pair(24, 32, 42, False)
    Xj = pair.Xji.astype(np.float64).copy()
    Xj[0, 0] = [np.nan, 0, 1]
    Xj[1, 1] = [0, 0, 0]
    Xj[2, 2] = [np.inf, 1, 1]
    Xi = pair.Xii.astype(np.float64).copy()
    Xi[20, 30] = [np.nan, np.nan, np.nan]
    pinit = np.stack(synth.pixel_grid(24, 32), -1).astype(np.float64)
    pinit[3, 3] = [np.nan, 1.0]
    o = fwd(lib, Xi, Xj, p_init=pinit)
    for (y, x) in [(0, 0), (1, 1), (2, 2), (3, 3)]:
        assert o["idx"][y, x] == -1 and not o["valid"][y, x] and o["theta"][y, x] == np.inf
    ref = fwd(lib, pair.Xii, pair.Xji)
    far = np.ones((24, 32), bool)
    far[14:, 22:] = False
    far[:4, :4] = False
    assert np.array_equal(o["p"][far], ref["p"][far]), "bad reference pixel leaked"
    assert np.isfinite(o["p"]).all()


def pin_p_init(lib):
    """Initialisation from given pixels (Sec. 3.2, tracking): starting at the pinhole
    projection, or a few pixels away from it, converges to the same match."""
    pair = _pair(48, 64, 1001, False)
    ref = fwd(lib, pair.Xii, pair.Xji)
    m = ref["valid"] & _interior_true_match(pair, 1.0)
    o1 = fwd(lib, pair.Xii, pair.Xji, p_init=pair.proj)
    o2 = fwd(lib, pair.Xii, pair.Xji, p_init=pair.proj + 2.5)
    assert np.abs(o1["p"] - ref["p"])[m].max() <= 1e-9
    assert np.abs(o2["p"] - ref["p"])[m].max() <= 1e-9


def _position_code(xs, ys, n_dir=16, omega=0.04):
    """Unit descriptors whose dot product sum_k cos(omega u_k . (a - b)) / n_dir
    is isotropic and falls monotonically with pixel distance up to ~2.4/omega."""
    ang = np.arange(n_dir) * np.pi / n_dir
    u = np.stack([np.cos(ang), np.sin(ang)], -1)
    ph = omega * (np.asarray(xs)[..., None] * u[:, 0] + np.asarray(ys)[..., None] * u[:, 1])
    return np.concatenate([np.cos(ph), np.sin(ph)], -1) / np.sqrt(n_dir)


def pin_refine_coarse_to_fine(lib):
    """Coarse-to-fine refine (Sec. 3.2): with a similarity that falls with pixel
    distance, L levels of spacing 2^(L-1)..1 and radius r land exactly on a
    target up to r (2^L - 1) px from the rounded match; one level cannot reach
    beyond r."""
    pair = _pair(96, 128, 21, False)
    H, W = pair.H, pair.W
    base = fwd(lib, pair.Xii, pair.Xji, pair.Dii, pair.Dji)
    m0 = np.floor(base["p"] + 0.5).astype(int)
    xs, ys = synth.pixel_grid(H, W)
    Dii = _position_code(xs, ys)
    rng = np.random.Generator(np.random.PCG64(4))
    r = 3
    for L in (2, 3):
        reach = r * (2 ** L - 1) - 1
        off = rng.integers(-reach, reach + 1, size=(H, W, 2))
        tx = m0[..., 0] + off[..., 0]
        ty = m0[..., 1] + off[..., 1]
        ok = (tx >= 0) & (tx < W) & (ty >= 0) & (ty < H) & base["valid"]
        Dji = _position_code(tx, ty)
        o = fwd(lib, pair.Xii, pair.Xji, Dii, Dji, r=r, levels=L)
        want = ty * W + tx
        assert ok.sum() > 1000
        assert (o["idx"][ok] == want[ok]).all(), "coarse-to-fine with %d levels" % L
        far = ok & (np.abs(off).max(-1) > r)
        o1 = fwd(lib, pair.Xii, pair.Xji, Dii, Dji, r=r, levels=1)
        assert far.sum() > 100 and not (o1["idx"][far] == want[far]).any(), "one level reaches only r"
    one = fwd(lib, pair.Xii, pair.Xji, pair.Dii, pair.Dji, r=r, levels=1)
    assert np.array_equal(one["idx"], base["idx"]), "one level is the plain window"


def pin_match_stats(lib):
    """Keyframe statistics (Sec. 3.4): valid count and distinct matched reference
    pixels, on cases with known answers."""
    p = synth.identity_pair(12, 16, 3)
    o = fwd(lib, p.Xii, p.Xji, p.Dii, p.Dji)
    assert oracle.match_stats(o["idx"], o["valid"]) == (192, 192)
    idx = np.full((12, 16), 7, np.int32)
    valid = np.zeros((12, 16), bool)
    valid[:3] = True
    assert oracle.match_stats(idx, valid) == (48, 1)
    idx2 = np.arange(192, dtype=np.int32).reshape(12, 16) // 2
    assert oracle.match_stats(idx2, np.ones((12, 16), bool)) == (192, 96)


# --------------------------------------------------------------- tracking pins

def _sim3_generator_expm(tau):
    import scipy.linalg as sl
    v, w, s = tau[:3], tau[3:6], tau[6]
    S = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    M = np.zeros((4, 4))
    M[:3, :3] = S + s * np.eye(3)
    M[:3, 3] = v
    return sl.expm(M)[:3]


def pin_sim3_exp(lib):
    """Exp of sim(3) (Eq. 1) equals the matrix exponential of the 4x4 generator
    [[[omega]_x + sigma I, v], [0, 0]], including near theta = 0 and sigma = 0."""
    rng = np.random.Generator(np.random.PCG64(12))
    for scale in (1e-9, 1e-6, 1e-4, 1e-3, 1e-2, 0.3, 1.5):
        for _ in range(10):
            tau = rng.normal(size=7) * scale
            assert np.abs(oracle.sim3_exp(tau, lib) - _sim3_generator_expm(tau)).max() <= 1e-10, "Exp at %g" % scale
    for tau in ([0.1, 0.2, 0.3, 1e-5, 0, 0, 0.2], [0.1, 0.2, 0.3, 0.5, 0.1, 0, 1e-5], [0.1, -0.2, 0.3, 0, 0, 0, 0]):
        tau = np.array(tau)
        assert np.abs(oracle.sim3_exp(tau, lib) - _sim3_generator_expm(tau)).max() <= 1e-10


def _compose(A, T):
    out = np.zeros((3, 4))
    out[:, :3] = A[:, :3] @ T[:, :3]
    out[:, 3] = A[:, :3] @ T[:, 3] + A[:, 3]
    return out


def pin_track_jacobians(lib):
    """Ray and distance Jacobians w.r.t. a left perturbation of the pose (Supp. A,
    Eq. point_jac, norm_jac, dist_jac) vs central differences of the residuals
    under Exp(eps e_k) o T."""
    rng = np.random.Generator(np.random.PCG64(13))
    for _ in range(20):
        T = oracle.sim3_exp(rng.normal(size=7) * 0.3, lib)
        Xf = rng.normal(size=3) + np.array([0, 0, 3.0])
        Xk = rng.normal(size=3) + np.array([0, 0, 3.0])
        r, J = oracle.track_residual(T, Xf, Xk, lib)
        eps = 1e-6
        for k in range(7):
            e = np.zeros(7); e[k] = eps
            rp, _ = oracle.track_residual(_compose(oracle.sim3_exp(e, lib), T), Xf, Xk, lib)
            rm, _ = oracle.track_residual(_compose(oracle.sim3_exp(-e, lib), T), Xf, Xk, lib)
            fd = (rp - rm) / (2 * eps)
            assert np.abs(fd - J[:, k]).max() <= 1e-7 * max(1.0, np.abs(J).max()), "Jacobian column %d" % k
    # The ray residual does not depend on the scale (psi is depth invariant).
    assert (J[:3, 6] == 0).all()


def pin_track_recovers_pose(lib):
    """Noise-free matches: 10 Gauss-Newton iterations from the identity recover
    the true Sim(3) (Eq. gauss_newton with the left-plus update of Eq. 1)."""
    for seed in (1, 2, 3):
        tp = synth.make_tracking(24, 32, seed)
        T0 = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
        T, info = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk, T0, lib=lib)
        err = np.abs(T - tp.T_true).max()
        assert info["solved"] == 10 and err <= 1e-6, "pose error %g" % err
        assert np.abs(info["g"]).max() <= 1e-6 * max(1.0, np.abs(info["H"]).max())
    # A large motion (90 deg, unit translation, scale 1.6) started near the truth:
    # the step is a left perturbation, so it must be applied on the left.
    tp = synth.make_tracking(24, 32, 9, max_deg=90.0, max_t=1.0, scale_range=(1.5, 1.7))
    rng = np.random.Generator(np.random.PCG64(9))
    T0 = _compose(oracle.sim3_exp(rng.normal(size=7) * 0.02, lib), tp.T_true)
    T, info = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk, T0, iters=6, lib=lib)
    assert np.abs(T - tp.T_true).max() <= 1e-6, "large-motion pose error %g" % np.abs(T - tp.T_true).max()


def pin_track_distance_term(lib):
    """Sec. 3.3: the ray residual alone leaves scale unobservable (its scale column
    is zero), so the system is singular; the distance term makes it solvable,
    also under pure rotation."""
    tp = synth.make_tracking(24, 32, 4, pure_rotation=True)
    T0 = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    _, info = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk, T0, sigma_dist=math.inf, lib=lib)
    assert info["solved"] == 0, "ray-only system must be singular"
    T, info = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk, T0, lib=lib)
    assert info["solved"] == 10 and np.abs(T - tp.T_true).max() <= 1e-6


def pin_track_robust(lib):
    """Huber weights (Sec. 3.3) bound the influence of gross outliers: with 20 %
    displaced matches the robust pose is far closer to the truth than the
    least-squares one; giving the outliers confidences below q_min removes them."""
    tp = synth.make_tracking(24, 32, 5, noise=1e-3, outlier_frac=0.2)
    T0 = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    Tr, _ = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk, T0, iters=20, lib=lib)
    Tl, _ = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk, T0, iters=20, huber=math.inf, lib=lib)
    er, el = np.abs(Tr - tp.T_true).max(), np.abs(Tl - tp.T_true).max()
    assert er < 0.2 * el, "robust %g vs least squares %g" % (er, el)
    Qk = tp.Qk.copy()
    Qk[tp.outlier] = 0.25                 # q = sqrt(Qf Qk) <= sqrt(5 * 0.25) < 1.5
    tp_clean = synth.make_tracking(24, 32, 5, noise=0.0, outlier_frac=0.2)
    Qk2 = tp_clean.Qk.copy()
    Qk2[tp_clean.outlier] = 0.25
    Tg, _ = oracle.track_pose(tp_clean.Xk, tp_clean.Xf, tp_clean.idx, tp_clean.valid, tp_clean.Qf, Qk2, T0,
                              huber=math.inf, lib=lib)
    assert np.abs(Tg - tp_clean.T_true).max() <= 1e-6, "confidence gate"


def pin_track_confidence_weight(lib):
    """The per-match weight is q / sigma^2 (Sec. 3.3, w(q, sigma^2) = sigma^2 / q):
    one match of confidence 2q acts exactly like two identical matches of
    confidence q.  Two groups of matches with different noise pull the pose
    differently, so a weight not linear in q changes the result."""
    H, W = 16, 32
    tp = synth.make_tracking(H, W // 2, 8, noise=2e-2, valid_frac=1.0)
    Xk = np.concatenate([tp.Xk, tp.Xk], 1)
    Xf = tp.Xf
    Xf2 = np.concatenate([Xf, Xf], 1)
    idx_half = tp.idx
    ys = np.arange(H)[:, None]
    # Remap frame indices from the (H, W/2) frame to the (H, W) frame (left half).
    idx_l = (idx_half // (W // 2)) * W + idx_half % (W // 2)
    idx = np.concatenate([idx_l, idx_l], 1).astype(np.int32)
    group2 = (np.arange(W // 2)[None, :] >= W // 4) & np.ones((H, 1), bool)
    T0 = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    # A: left half only; group 1 with q = 2, group 2 with q = 4.
    Qf = np.full((H, W), 2.0)
    QkA = np.concatenate([np.where(group2, 8.0, 2.0), np.ones((H, W // 2))], 1)
    validA = np.concatenate([np.ones((H, W // 2), bool), np.zeros((H, W // 2), bool)], 1)
    # B: both halves; every match with q = 2, group 2 duplicated in the right half.
    QkB = np.full((H, W), 2.0)
    validB = np.concatenate([np.ones((H, W // 2), bool), group2], 1)
    kw = dict(q_min=0.5, huber=math.inf, iters=15, lib=lib)
    TA, _ = oracle.track_pose(Xk, Xf2, idx, validA, Qf, QkA, T0, **kw)
    TB, _ = oracle.track_pose(Xk, Xf2, idx, validB, Qf, QkB, T0, **kw)
    TC, _ = oracle.track_pose(Xk, Xf2, idx, validA, Qf, np.full((H, W), 2.0), T0, **kw)
    assert np.abs(TA - TB).max() <= 1e-9, "weight must be linear in q"
    assert np.abs(TA - TC).max() > 1e-5, "the two groups must pull the pose apart"


# --------------------------------------------------------------- backward pins

def _fd_setup(lib, K=20):
    pair = _pair(24, 32, 5000)
    o = fwd(lib, pair.Xii, pair.Xji, K=K)
    frac = o["p"] - np.floor(o["p"])
    near_edge = ((frac < 1e-5) | (frac > 1 - 1e-5)).any(-1)
    mask = o["valid"] & ~near_edge
    return pair, o, mask


def _loss(lib, Xii, Xji, mask, K=20):
    o = fwd(lib, Xii, Xji, K=K)
    d = o["xhat"] - Xji
    return float((d * d).sum(-1)[mask].sum())


def _adjoint_total(lib, pair, o, mask):
    Xi = pair.Xii.astype(np.float64)
    Xj = pair.Xji.astype(np.float64)
    gx = 2.0 * (o["xhat"] - Xj) * mask[..., None]
    dXi, dXj = oracle.match_bwd(Xi, Xj, o["p"], mask, None, gx, lib=lib)
    return dXi, dXj - gx


def pin_bwd_fd(lib):
    """Implicit adjoint vs central finite differences (eps 1e-6, fp64, mask frozen,
    queries within 1e-5 px of a bilinear cell edge left out) on a 32x24 pair."""
    pair, o, mask = _fd_setup(lib)
    gi, gj = _adjoint_total(lib, pair, o, mask)
    Xi = pair.Xii.astype(np.float64)
    Xj = pair.Xji.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(8))
    eps = 1e-6
    for name, X, G in (("Xii", Xi, gi), ("Xji", Xj, gj)):
        flat = rng.choice(X.size, size=120, replace=False)
        # Always include the largest-gradient elements.
        flat = np.unique(np.concatenate([flat, np.argsort(-np.abs(G).reshape(-1))[:30]]))
        scale = np.abs(G).max()
        for e in flat:
            Xp = X.copy(); Xp.reshape(-1)[e] += eps
            Xm = X.copy(); Xm.reshape(-1)[e] -= eps
            if name == "Xii":
                fd = (_loss(lib, Xp, Xj, mask) - _loss(lib, Xm, Xj, mask)) / (2 * eps)
            else:
                fd = (_loss(lib, Xi, Xp, mask) - _loss(lib, Xi, Xm, mask)) / (2 * eps)
            g = G.reshape(-1)[e]
            assert abs(fd - g) <= 1e-5 * max(abs(fd), 1e-2 * scale), \
                "FD %s[%d]: fd %.10g adjoint %.10g" % (name, e, fd, g)


def pin_bwd_unrolled(lib):
    """Implicit adjoint vs torch fp64 autograd through the unrolled iterations of an
    independent statement of the solver (20 iterations, converged)."""
    import torch
    from oracle import unrolled
    pair, o, mask = _fd_setup(lib)
    Xi = torch.tensor(pair.Xii, dtype=torch.float64, requires_grad=True)
    Xj = torch.tensor(pair.Xji, dtype=torch.float64, requires_grad=True)
    p, th, xh = unrolled.lm_project(Xi, Xj, K=20)
    dp = np.abs(p.detach().numpy().reshape(o["p"].shape) - o["p"]).max(-1)
    # Converged (valid) queries agree to rounding.  Queries beyond the image
    # border are held on it and still step along it after 20 iterations, so
    # the two fp64 statements' different operation orders leave a few 1e-9 px
    # there; every query is pinned, those at 1e-7 px.
    assert dp[o["valid"]].max() <= 1e-9, "unrolled p*"
    assert dp.max() <= 1e-7, "unrolled p* (all queries)"
    m = torch.tensor(mask.reshape(-1))
    L = ((xh - Xj.reshape(-1, 3)) ** 2).sum(-1)[m].sum()
    L.backward()
    gi, gj = _adjoint_total(lib, pair, o, mask)
    assert np.abs(gi - Xi.grad.numpy()).max() <= 1e-8 * np.abs(gi).max(), "unrolled dXii"
    assert np.abs(gj - Xj.grad.numpy()).max() <= 1e-8 * np.abs(gj).max(), "unrolled dXji"


def pin_bwd_orthogonal(lib):
    """Through the ray map only (no xhat gradient) the adjoint is orthogonal to the
    radial direction: N(X) = (I - u u^T)/|X| annihilates X (Supp. A, Eq. norm_jac)."""
    pair, o, mask = _fd_setup(lib)
    rng = np.random.Generator(np.random.PCG64(1))
    gp = rng.normal(size=o["p"].shape)
    Xi = pair.Xii.astype(np.float64)
    Xj = pair.Xji.astype(np.float64)
    dXi, dXj = oracle.match_bwd(Xi, Xj, o["p"], mask, gp, None, lib=lib)
    rad_i = (dXi * Xi).sum(-1) / np.linalg.norm(Xi, axis=-1)
    rad_j = (dXj * Xj).sum(-1) / np.linalg.norm(Xj, axis=-1)
    assert np.abs(rad_i).max() <= 1e-12 * np.abs(dXi).max()
    assert np.abs(rad_j).max() <= 1e-12 * np.abs(dXj).max()
    assert (dXj[~mask] == 0).all(), "invalid queries contribute nothing"
    assert np.abs(dXj[mask]).max() > 0


def pin_bwd_projection_jacobian(lib):
    """For a pinhole ray image, dp*/dx is the pinhole projection Jacobian
    (f/z) [[1, 0, -x/z], [0, 1, -y/z]] (Supp. A, projection Jacobian), up to the
    interpolation error of the ray image."""
    pair = _pair(120, 160, 77, False)
    o = fwd(lib, pair.Xii, pair.Xji)
    m = o["valid"] & _interior_true_match(pair, 1.0)
    f, cx, cy = synth.camera(pair.H, pair.W)
    X = pair.Xji.astype(np.float64)
    x, y, z = X[..., 0], X[..., 1], X[..., 2]
    for comp in (0, 1):
        gp = np.zeros(o["p"].shape)
        gp[..., comp] = 1.0
        _, dXj = oracle.match_bwd(pair.Xii, X, o["p"], m, gp, None, lib=lib)
        want = np.zeros_like(X)
        want[..., comp] = f / z
        want[..., 2] = -f * (x if comp == 0 else y) / z ** 2
        err = np.linalg.norm(dXj - want, axis=-1)[m] / np.linalg.norm(want, axis=-1)[m]
        assert err.max() <= 5e-2, "projection Jacobian row %d: %g" % (comp, err.max())


def pin_bwd_held_border(lib):
    """Matches held on the image border (their rays lie just outside it): the
    held coordinate does not move and the other one follows its 1-D system.
    Central finite differences of the loss through the forward agree with the
    adjoint to the Gauss-Newton approximation error at a small residual (the
    adjoint of a free coordinate would be off by far more)."""
    H, W = 24, 32
    R, f, cx, cy = pinhole_rays(H, W)
    xs, ys = synth.pixel_grid(H, W)
    z = 2.0 + 0.2 * np.sin(0.3 * xs) * np.cos(0.2 * ys)
    Xii = R * z[..., None]
    Xj = np.tile(np.array([0.0, 0.0, 1.0]), (H, W, 1)) * 2.0
    queries = []
    for k, yq in enumerate([3.3, 7.6, 12.2, 17.9]):       # beyond the right border
        u, v = (W - 1 + 2e-4 - cx) / f, (yq - cy) / f
        Xj[2 + 4 * k, 4] = np.array([u, v, 1.0]) * (1.5 + 0.1 * k)
        queries.append((2 + 4 * k, 4, 0))
    for k, xq in enumerate([5.4, 11.7, 20.1]):             # beyond the bottom border
        u, v = (xq - cx) / f, (H - 1 + 2e-4 - cy) / f
        Xj[3 + 4 * k, 9] = np.array([u, v, 1.0]) * (1.8 - 0.1 * k)
        queries.append((3 + 4 * k, 9, 1))
    mask = np.zeros((H, W), bool)
    for (y, x, _) in queries:
        mask[y, x] = True
    K = 20
    o = fwd(lib, Xii, Xj, K=K, max_theta=math.inf)
    for (y, x, ax) in queries:
        assert o["p"][y, x, ax] == (W - 1 if ax == 0 else H - 1), "held match not on the border"

    def loss(Xi_, Xj_):
        oo = fwd(lib, Xi_, Xj_, K=K, max_theta=math.inf)
        d = oo["xhat"] - Xj_
        return float((d * d).sum(-1)[mask].sum())

    gx = 2.0 * (o["xhat"] - Xj) * mask[..., None]
    dXi, dXj = oracle.match_bwd(Xii, Xj, o["p"], mask, None, gx, lib=lib)
    dXj = dXj - gx
    eps = 1e-6
    checks = [("Xji", (y, x, c)) for (y, x, _) in queries for c in range(3)]
    checks += [("Xii", (y, W - 1, c)) for y in range(2, 20, 3) for c in range(3)]
    checks += [("Xii", (H - 1, x, c)) for x in range(4, 22, 3) for c in range(3)]
    scale = max(np.abs(dXi).max(), np.abs(dXj).max())
    for name, ix in checks:
        A = Xii if name == "Xii" else Xj
        Ap = A.copy(); Ap[ix] += eps
        Am = A.copy(); Am[ix] -= eps
        if name == "Xii":
            fd = (loss(Ap, Xj) - loss(Am, Xj)) / (2 * eps)
            g = dXi[ix]
        else:
            fd = (loss(Xii, Ap) - loss(Xii, Am)) / (2 * eps)
            g = dXj[ix]
        assert abs(fd - g) <= 2e-3 * max(abs(fd), 0.05 * scale), \
            "held border FD %s%s: fd %.8g adjoint %.8g" % (name, ix, fd, g)


def pin_fuse_sequence_is_weighted_mean(lib):
    """Eq. 8 folded over several frames is the confidence-weighted mean of the
    transformed points, with the confidences summed (a closed form that
    involves no running update), and a zero-confidence start returns T X."""
    H, W = 12, 16
    rng = np.random.Generator(np.random.PCG64(77))
    P = rng.normal(size=(H * W, 3)) + np.array([0.0, 0.0, 3.0])
    Xc = np.zeros((H * W, 3))
    Cc = np.zeros(H * W)
    num = np.zeros((H * W, 3))
    den = np.zeros(H * W)
    for k in range(4):
        s, R, t = synth.random_sim3(rng, 30.0, 0.5, 0.7, 1.4)
        T = np.concatenate([s * R, t[:, None]], 1)
        Pk = P + rng.normal(0.0, 0.05, size=P.shape)
        X = ((Pk - t) @ R) / s                     # the frame sees Pk through T^-1
        C = rng.uniform(0.1, 5.0, size=H * W)
        Xc, Cc = oracle.fuse(T, Xc, Cc, X, C, lib=lib)
        num += C[:, None] * Pk
        den += C
        if k == 0:
            assert np.abs(Xc - Pk).max() < 1e-12, "fusion into an empty map must give T X"
    assert np.abs(Cc - den).max() < 1e-12
    assert np.abs(Xc - num / den[:, None]).max() < 1e-12


def pin_fuse_degenerate(lib):
    """Zero new confidence keeps the map; zero summed confidence keeps the point."""
    fp = synth.make_fusion(8, 10, 5)
    C0 = np.zeros_like(fp.C, dtype=np.float64)
    Xc, Cc = oracle.fuse(fp.T, fp.Xc, fp.Cc, fp.X, C0, lib=lib)
    assert np.array_equal(Xc, fp.Xc.astype(np.float64)) and np.array_equal(Cc, fp.Cc.astype(np.float64))
    Xc, Cc = oracle.fuse(fp.T, fp.Xc, np.zeros_like(Cc), fp.X, C0, lib=lib)
    assert np.array_equal(Xc, fp.Xc.astype(np.float64)) and not Cc.any()
    # Equal confidences: the midpoint of the old point and the transformed new one.
    Xc, Cc = oracle.fuse(fp.T, fp.Xc, np.ones_like(Cc), fp.X, np.ones_like(Cc), lib=lib)
    TX, _ = oracle.fuse(fp.T, np.zeros_like(fp.Xc), np.zeros_like(Cc), fp.X, np.ones_like(Cc), lib=lib)
    assert np.abs(Xc - 0.5 * (fp.Xc + TX)).max() < 1e-12 and np.all(Cc == 2.0)
    # T X is the keyframe-frame point up to the generator's noise (0.01 per axis).
    assert np.abs(TX - fp.P).max() < 0.1


def _sim3_rand(rng, deg=20.0, tmax=0.5, smin=0.7, smax=1.4):
    s, R, t = synth.random_sim3(rng, deg, tmax, smin, smax)
    return np.concatenate([s * R, t[:, None]], 1)


def _pose_gap(A, B):
    """Largest entry-wise difference of two 3x4 poses."""
    return float(np.abs(np.asarray(A) - np.asarray(B)).max())


def pin_backend_jacobians(lib):
    """Central differences of the backend residuals under left perturbations
    Exp(eps e_k) T of each world pose match the analytic Jacobians (Supp. A,
    relative-to-global chain rule); the residuals depend on T_i^-1 T_j only."""
    rng = np.random.Generator(np.random.PCG64(31))
    for trial in range(4):
        Ti, Tj = _sim3_rand(rng), _sim3_rand(rng)
        Xj = rng.normal(size=3) + np.array([0.0, 0.0, 3.0])
        Xi = rng.normal(size=3) + np.array([0.0, 0.0, 3.0])
        r, Ji, Jj = oracle.backend_residual(Ti, Tj, Xj, Xi, lib=lib)
        eps = 1e-6
        for which, J in (("i", Ji), ("j", Jj)):
            for k in range(7):
                tau = np.zeros(7)
                tau[k] = eps
                Ep, Em = oracle.sim3_exp(tau, lib=lib), oracle.sim3_exp(-tau, lib=lib)
                if which == "i":
                    rp = oracle.backend_residual(_compose(Ep, Ti), Tj, Xj, Xi, lib=lib)[0]
                    rm = oracle.backend_residual(_compose(Em, Ti), Tj, Xj, Xi, lib=lib)[0]
                else:
                    rp = oracle.backend_residual(Ti, _compose(Ep, Tj), Xj, Xi, lib=lib)[0]
                    rm = oracle.backend_residual(Ti, _compose(Em, Tj), Xj, Xi, lib=lib)[0]
                fd = (rp - rm) / (2 * eps)
                assert np.abs(fd - J[:, k]).max() <= 1e-6 * max(1.0, np.abs(J).max()), \
                    "backend J_%s column %d: fd %s analytic %s" % (which, k, fd, J[:, k])
        # A common world transform G leaves the residuals unchanged.
        G = _sim3_rand(rng)
        r2 = oracle.backend_residual(_compose(G, Ti), _compose(G, Tj), Xj, Xi, lib=lib)[0]
        assert np.abs(r2 - r).max() < 1e-12


def pin_backend_two_keyframes_is_tracking(lib):
    """Two keyframes with the first held at a pose G and pixel-aligned matches:
    each backend step on T_WC1 is the tracking step on T_01 = G^-1 T_WC1
    carried by Ad(G), so the backend ends at G times the tracking result."""
    bp = synth.make_backend(2, 12, 16, 41, scramble=False, noise=1e-3, loops=0)
    rng = np.random.Generator(np.random.PCG64(42))
    G = _sim3_rand(rng)
    T0 = np.stack([G, _compose(G, bp.T_init[1])])
    edges = np.array([[0, 1]], np.int32)
    idx = np.arange(12 * 16, dtype=np.int32).reshape(1, 12, 16)
    valid = bp.valid[:1]
    T_b, info = oracle.backend_gn(bp.Xc, bp.Q, edges, idx, valid, T0, iters=6, lib=lib)
    T_t, tinfo = oracle.track_pose(bp.Xc[0], bp.Xc[1], idx[0], valid[0], bp.Q[1], bp.Q[0], bp.T_init[1],
                                   iters=6, lib=lib)
    assert np.array_equal(T_b[0], T0[0]), "the gauge keyframe moved"
    assert _pose_gap(T_b[1], _compose(G, T_t)) < 1e-9, _pose_gap(T_b[1], _compose(G, T_t))
    assert info["count"] == tinfo["count"] and abs(info["cost"] - tinfo["cost"]) <= 1e-9 * max(tinfo["cost"], 1.0)


def pin_backend_recovers_poses(lib):
    """Noise-free keyframe chain with a loop closure and scrambled pixel
    correspondences: from perturbed poses, Gauss-Newton reaches the generating
    poses; a world transform of the start transforms the result (gauge)."""
    bp = synth.make_backend(5, 10, 12, 43, scramble=True, loops=1)
    T, info = oracle.backend_gn(bp.Xc, bp.Q, bp.edges, bp.idx, bp.valid, bp.T_init, iters=12, lib=lib)
    assert np.array_equal(T[0], bp.T_init[0])
    for k in range(bp.N):
        assert _pose_gap(T[k], bp.T_true[k]) < 2e-6, (k, _pose_gap(T[k], bp.T_true[k]))
    assert info["last_step"] < 1e-6 and info["applied"] == 12
    G = _sim3_rand(np.random.Generator(np.random.PCG64(44)))
    TG = np.stack([_compose(G, t) for t in bp.T_init])
    T2, _ = oracle.backend_gn(bp.Xc, bp.Q, bp.edges, bp.idx, bp.valid, TG, iters=12, lib=lib)
    for k in range(bp.N):
        assert _pose_gap(T2[k], _compose(G, T[k])) < 1e-8
    # Early exit: a step tolerance stops the loop once the steps are small.
    T3, info3 = oracle.backend_gn(bp.Xc, bp.Q, bp.edges, bp.idx, bp.valid, bp.T_init, iters=50, step_tol=1e-9,
                                  lib=lib)
    assert info3["applied"] < 50 and info3["last_step"] < 1e-9


def pin_backend_robust(lib):
    """Noise and 10 % gross outliers: the Huber-weighted solve stays close to
    the generating poses, and the plain least-squares solve does worse."""
    bp = synth.make_backend(4, 16, 20, 45, scramble=True, noise=1e-3, outlier_frac=0.1, loops=1)
    T, _ = oracle.backend_gn(bp.Xc, bp.Q, bp.edges, bp.idx, bp.valid, bp.T_init, iters=10, lib=lib)
    Tl, _ = oracle.backend_gn(bp.Xc, bp.Q, bp.edges, bp.idx, bp.valid, bp.T_init, iters=10, huber=float("inf"),
                              lib=lib)
    err = max(_pose_gap(T[k], bp.T_true[k]) for k in range(bp.N))
    err_ls = max(_pose_gap(Tl[k], bp.T_true[k]) for k in range(bp.N))
    assert err < 5e-3, err
    assert err_ls > 2 * err, (err, err_ls)


ALL_PINS = [
    pin_identity, pin_pinhole, pin_brute_force, pin_depth_invariance, pin_border_angle,
    pin_gradient_images, pin_convergence, pin_refine_planted, pin_refine_ties, pin_conf_gate,
    pin_dist_gate, pin_theta_gate, pin_bad_inputs, pin_p_init, pin_refine_coarse_to_fine, pin_match_stats,
    pin_bwd_fd, pin_bwd_unrolled, pin_bwd_orthogonal, pin_bwd_projection_jacobian, pin_bwd_held_border,
    pin_sim3_exp, pin_track_jacobians, pin_track_recovers_pose, pin_track_distance_term, pin_track_robust,
    pin_track_confidence_weight, pin_fuse_sequence_is_weighted_mean, pin_fuse_degenerate,
    pin_backend_jacobians, pin_backend_two_keyframes_is_tracking, pin_backend_recovers_poses, pin_backend_robust,
]
