"""GPU parity of the tracking pose solve (Sec. 3.3) against the fp64 oracle.

Both sides take the same seeded synthetic problem (frame points on the
procedural surface, a random Sim(3), matches that shift pixels, optional noise
and gross outliers) and the same initial pose.

Tolerance (derived from the arithmetic, not fitted): the library evaluates
residuals and Jacobians in fp32 from fp32 points and sums the normal equations
in fp32 per workgroup, fp64 across.  The fixed point of Gauss-Newton moves by
H^-1 J^T W dr, where dr is the rounding error of the residual: a few ulps of a
unit ray (<= 3e-7) and of a distance near 2 (<= 5e-7).  A systematic error of
that size moves the rotation by <= 3e-7 rad and the translation by <= 1e-6 of
the scene depth; the fp32 summation of g adds a random error far below that
(relative 6e-8 per term, H ~ 1e9).  The test allows 1e-5 rad, 2e-5 in
translation and 1e-5 in log-scale: a margin of about 30 over the bound, and far
below what a wrong term changes (a dropped distance term or a sign error moves
the pose by more than 1e-3).  The confidence gate is decided in fp64 on both
sides, so the match count and the number of solved iterations are exact.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2412_12392_amd import track_params, track_pose

pytestmark = pytest.mark.gpu

ROT_TOL = 1e-5
T_TOL = 2e-5
S_TOL = 1e-5


def _to_dev(tp):
    d = "cuda:0"
    return (torch.from_numpy(tp.Xk).to(d), torch.from_numpy(tp.Xf).to(d),
            torch.from_numpy(tp.idx.astype(np.int32)).to(d),
            torch.from_numpy(tp.valid.astype(np.uint8)).to(d),
            torch.from_numpy(tp.Qf).to(d), torch.from_numpy(tp.Qk).to(d))


def _pose_diff(Ta, Tb):
    """(rotation angle, translation distance, |log scale ratio|) between two 3x4 Sim(3)."""
    Ta, Tb = np.asarray(Ta, np.float64), np.asarray(Tb, np.float64)
    sa = np.cbrt(np.linalg.det(Ta[:, :3]))
    sb = np.cbrt(np.linalg.det(Tb[:, :3]))
    R = (Ta[:, :3] / sa) @ (Tb[:, :3] / sb).T
    ang = np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1))
    return ang, np.linalg.norm(Ta[:, 3] - Tb[:, 3]), abs(np.log(sa / sb))


def _run(tp, T0, **kw):
    args = dict(oracle.TRACK_DEFAULTS)
    args.update(kw)
    dev = _to_dev(tp)
    T = torch.tensor(np.asarray(T0, np.float32), device="cuda:0").contiguous()
    prm = track_params(**args)
    _, info = track_pose(*dev, T, prm)
    torch.cuda.synchronize()
    T_ref, ref = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk,
                                   np.asarray(T0, np.float32).astype(np.float64), **args)
    return T.cpu().numpy(), info.cpu().numpy(), T_ref, ref


def _check(T, info, T_ref, ref, cost_rel=2e-3):
    ang, dt, ds = _pose_diff(T, T_ref)
    assert ang <= ROT_TOL and dt <= T_TOL and ds <= S_TOL, (ang, dt, ds)
    assert int(info[1]) == ref["count"]
    assert int(info[2]) == ref["solved"]
    if cost_rel is not None:
        assert abs(info[0] - ref["cost"]) <= cost_rel * ref["cost"] + 1e-6 * max(ref["count"], 1), (info[0], ref["cost"])


I34 = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)

CASES = [
    # name, (H, W, seed), make_tracking kwargs, solve kwargs, compare cost
    ("clean_small", (24, 32, 1), {}, {}, False),
    ("noise_outliers", (48, 64, 2), dict(noise=1e-3, outlier_frac=0.1), {}, True),
    ("ragged", (37, 53, 3), dict(noise=5e-4, outlier_frac=0.05, valid_frac=0.7), {}, True),
    ("pure_rotation", (40, 56, 4), dict(pure_rotation=True, noise=1e-3), {}, True),
    ("no_distance", (32, 48, 5), dict(noise=1e-3), dict(sigma_dist=float("inf")), True),
    ("plain_least_squares", (32, 48, 6), dict(noise=1e-3), dict(huber=float("inf")), True),
    ("full_512x384", (384, 512, 7), dict(noise=1e-3, outlier_frac=0.1), {}, True),
    ("many_blocks", (1024, 1280, 8), dict(noise=1e-3, outlier_frac=0.05), dict(iters=4), True),
    # More matches than the accumulation grid covers in one stride (2048 workgroups x 1024).
    ("beyond_grid", (1536, 1536, 15), dict(noise=1e-3, outlier_frac=0.05), dict(iters=3), True),
]


@pytest.mark.parametrize("name,shape,gen,solve,cmp_cost", CASES, ids=[c[0] for c in CASES])
def test_track_matches_oracle(name, shape, gen, solve, cmp_cost):
    H, W, seed = shape
    print("track case", name, H, W, seed, flush=True)
    tp = synth.make_tracking(H, W, seed, **gen)
    T, info, T_ref, ref = _run(tp, I34, **solve)
    _check(T, info, T_ref, ref, 2e-3 if cmp_cost else None)
    if not cmp_cost:
        # Noise-free: both converge onto the true pose; the cost is rounding.
        assert info[0] <= 1e-3 * max(ref["count"], 1)
    # The solve itself must have reached the generating pose where there are no outliers.
    if gen.get("outlier_frac", 0.0) == 0.0 and gen.get("noise", 0.0) == 0.0:
        ang, dt, ds = _pose_diff(T, tp.T_true)
        assert ang < 1e-5 and dt < 1e-4 and ds < 1e-5


def test_track_large_motion():
    tp = synth.make_tracking(48, 64, 9, max_deg=60.0, max_t=0.5, scale_range=(0.8, 1.25), noise=1e-3)
    T, info, T_ref, ref = _run(tp, I34, iters=20)
    _check(T, info, T_ref, ref)


def test_track_zero_iterations_and_empty():
    tp = synth.make_tracking(24, 32, 10, noise=1e-3)
    T0 = np.array([[1.01, 0.0, 0.0, 0.02], [0.0, 1.01, 0.0, -0.01], [0.0, 0.0, 1.01, 0.03]], np.float32)
    T, info, T_ref, ref = _run(tp, T0, iters=0)
    assert np.array_equal(T, T0)
    assert int(info[2]) == 0 and int(info[1]) == ref["count"]
    assert abs(info[0] - ref["cost"]) <= 1e-3 * ref["cost"]
    # No valid match: singular system, every step skipped, pose unchanged.
    tp.valid[:] = False
    T, info, T_ref, ref = _run(tp, T0, iters=3)
    assert np.array_equal(T, T0) and int(info[1]) == 0 and int(info[2]) == 0 and info[0] == 0.0
    assert ref["solved"] == 0


def test_track_confidence_gate_exact():
    """Confidences on both sides of q_min by one fp32 ulp: the count is exact."""
    tp = synth.make_tracking(32, 48, 11, noise=1e-3)
    q = np.float32(1.5)
    n = tp.Qk.size
    Qf = np.full(n, q, np.float32)
    Qk = np.full(n, q, np.float32)
    Qk[::3] = np.nextafter(q, np.float32(2))
    Qk[1::3] = np.nextafter(q, np.float32(1))
    tp.Qf = Qf.reshape(tp.Qf.shape)
    tp.Qk = Qk.reshape(tp.Qk.shape)
    T, info, T_ref, ref = _run(tp, I34, q_min=1.5)
    _check(T, info, T_ref, ref)
    assert 0 < ref["count"] < int(tp.valid.sum())


def test_track_deterministic_and_graph():
    tp = synth.make_tracking(96, 128, 12, noise=1e-3, outlier_frac=0.1)
    dev = _to_dev(tp)
    T0 = torch.tensor(I34, dtype=torch.float32, device="cuda:0")
    prm = track_params()
    T_a = T0.clone()
    _, info_a = track_pose(*dev, T_a, prm)
    T_b = T0.clone()
    _, info_b = track_pose(*dev, T_b, prm)
    torch.cuda.synchronize()
    assert torch.equal(T_a, T_b) and torch.equal(info_a, info_b)

    # The whole solve is capturable: replay with fresh initial poses.
    T_g = T0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        track_pose(*dev, T_g, prm)          # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    T_g.copy_(T0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        _, info_g = track_pose(*dev, T_g, prm)
    for rep in range(3):
        T_g.copy_(T0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(T_g, T_a), rep
        assert torch.equal(info_g, info_a), rep
        # Eager work between replays.
        T_c = T0.clone()
        track_pose(*dev, T_c, prm)
        torch.cuda.synchronize()
        assert torch.equal(T_c, T_a)


# ---------------------------------------------------------------------------
# Canonical pointmap fusion (Eq. 8).
#
# Tolerance: the library transforms the point in fp32 (three products and
# three sums per coordinate), forms the weighted sum (two products, one sum)
# and divides through a reciprocal: at most about 8 fp32 roundings of the
# magnitudes involved, so |dXc| <= 8 u (|Xc| + sum_j |T_ij X_j| + |t_i|) with
# u = 2^-24.  The summed confidence is one fp32 addition of two fp32 values:
# it equals the fp64 sum rounded to fp32, bit for bit.

U32 = 2.0 ** -24


def _fuse_bound(T, Xc, X):
    T = np.asarray(T, np.float64)
    mag = np.abs(X.reshape(-1, 3)) @ np.abs(T[:, :3]).T + np.abs(T[:, 3])
    return 8 * U32 * (np.abs(Xc.reshape(-1, 3)) + mag)


def _dev_unaligned(a, offset):
    """A contiguous device copy of `a` starting `offset` floats into a buffer."""
    flat = torch.empty(a.size + offset, dtype=torch.float32, device="cuda:0")
    view = flat[offset:]
    view.copy_(torch.from_numpy(np.ascontiguousarray(a, np.float32).reshape(-1)))
    return view.view(a.shape)


@pytest.mark.parametrize("H,W,offset", [(2, 2, 0), (3, 5, 0), (37, 53, 0), (384, 512, 0), (37, 53, 1),
                                        (384, 512, 1)])
def test_fuse_matches_oracle(H, W, offset):
    from paper_2412_12392_amd import fuse_pointmap
    print("fuse case", H, W, offset, flush=True)
    fp = synth.make_fusion(H, W, 100 + H + offset)
    T32 = fp.T.astype(np.float32)
    Xc, Cc = _dev_unaligned(fp.Xc, offset), _dev_unaligned(fp.Cc, offset)
    X, C = _dev_unaligned(fp.X, offset), _dev_unaligned(fp.C, offset)
    T = torch.from_numpy(T32).to("cuda:0")
    fuse_pointmap(Xc, Cc, X, C, T)
    torch.cuda.synchronize()
    Xc_ref, Cc_ref = oracle.fuse(T32.astype(np.float64), fp.Xc, fp.Cc, fp.X, fp.C)
    got = Xc.cpu().numpy().reshape(-1, 3).astype(np.float64)
    err = np.abs(got - Xc_ref.reshape(-1, 3))
    bound = _fuse_bound(T32, fp.Xc, fp.X)
    assert np.all(err <= bound), float((err / bound).max())
    assert np.array_equal(Cc.cpu().numpy(), Cc_ref.astype(np.float32))
    # Pixels with no confidence on either side keep their point bit for bit.
    dead = (fp.Cc + fp.C).reshape(-1) == 0
    if dead.any():
        assert np.array_equal(got[dead], fp.Xc.reshape(-1, 3)[dead].astype(np.float64))


def test_track_then_fuse_on_device():
    """Pose solve and fusion chained on one stream, the pose never leaving the GPU."""
    from paper_2412_12392_amd import fuse_pointmap
    tp = synth.make_tracking(96, 128, 13, noise=1e-3, outlier_frac=0.05)
    fp = synth.make_fusion(96, 128, 14)
    dev = _to_dev(tp)
    T = torch.tensor(I34, dtype=torch.float32, device="cuda:0")
    track_pose(*dev, T, track_params())
    Xc, Cc = torch.from_numpy(fp.Xc).cuda(), torch.from_numpy(fp.Cc).cuda()
    fuse_pointmap(Xc, Cc, torch.from_numpy(fp.X).cuda(), torch.from_numpy(fp.C).cuda(), T)
    torch.cuda.synchronize()
    T_ref, _ = oracle.track_pose(tp.Xk, tp.Xf, tp.idx, tp.valid, tp.Qf, tp.Qk, I34, **oracle.TRACK_DEFAULTS)
    Xc_ref, Cc_ref = oracle.fuse(T_ref, fp.Xc, fp.Cc, fp.X, fp.C)
    # The two poses agree to the tracking tolerance; moved points near depth 3
    # then agree to about 3 ROT_TOL + T_TOL + 3 S_TOL < 1e-4.
    assert np.abs(Xc.cpu().numpy() - Xc_ref).max() < 1e-4
    assert np.array_equal(Cc.cpu().numpy(), Cc_ref.astype(np.float32))
