"""GPU forward parity: libm3s (fp32, gfx950) against the FP64 oracle, through the C ABI."""
import functools
import zlib
import math
import os

import numpy as np
import pytest

import oracle
import parity
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m3s():
    import paper_2412_12392_amd as m
    m.load_library()
    return m


@functools.lru_cache(maxsize=None)
def _pair(H, W, seed, conf=True):
    return synth.make_pair(H, W, seed, conf=conf)


def run(m3s, pair, p_init=None, want_xhat=True, **prm):
    t = parity.pair_tensors(pair)
    res = m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"],
                    parity.to_dev(p_init), m3s.params(**prm), want_theta=True, want_xhat=want_xhat)
    return parity.result_numpy(res)


def ora(pair, p_init=None, **kw):
    args = dict(oracle.DEFAULTS, K=pair.K, r=pair.r)
    args.update(kw)
    return oracle.match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji, p_init, **args)


def _prm_kw(kw):
    # oracle keyword -> library parameter name
    names = dict(K="max_iter", r="refine_radius", lambda0="lambda_init", conf_min="conf_min",
                 max_theta="max_theta", max_dist="max_dist", levels="refine_levels")
    return {names[k]: v for k, v in kw.items()}


def check(m3s, pair, label, p_init=None, p_theta_max=None, **kw):
    kw.setdefault("K", pair.K)
    kw.setdefault("r", pair.r)
    g = run(m3s, pair, p_init, **_prm_kw(kw))
    o = ora(pair, p_init, **kw)
    st = parity.compare(g, o, label, p_theta_max=p_theta_max, pair=pair, r=kw["r"], levels=kw.get("levels", 1))
    print(st)
    both = g["valid"] & o["valid"]
    if p_theta_max is not None:
        both &= o["theta"] <= p_theta_max
    if "xhat" in g and both.any():
        gx, ox = g["xhat"][both], o["xhat"][both]
        # NaN where the bilinear cell touches a non-finite reference point, on both sides.
        assert np.array_equal(np.isnan(gx), np.isnan(ox)), "xhat NaN pattern"
        fin = ~np.isnan(ox)
        if fin.any():
            assert np.abs(gx - ox)[fin].max() <= 1e-3 * max(1.0, np.abs(ox[fin]).max()), "xhat"
    return g, o, st


def test_config_64x48(m3s):
    """64x48 pair, identity init, 10 LM iterations, r = 3, no confidences."""
    pair = synth.config_pair(1)
    check(m3s, pair, "64x48")


def test_config_512x384(m3s):
    """512x384 pair with confidences gated at 1.5, 10 iterations, r = 3."""
    pair = synth.config_pair(2)
    _, _, st = check(m3s, pair, "512x384")
    assert st["idx_compared"] > 0.9 * st["valid_both"]


@pytest.mark.parametrize("H,W", [(2, 2), (3, 5), (37, 53), (129, 67), (5, 300), (300, 7)])
def test_ragged_shapes(m3s, H, W):
    """Shapes that are not multiples of any tile, down to the 2x2 minimum."""
    check(m3s, _pair(H, W, 31 * H + W), "%dx%d" % (H, W))


@pytest.mark.parametrize("H,W,r", [(40, 2, 0), (40, 2, 3), (2, 40, 0), (2, 40, 3), (3, 2, 1)])
def test_one_column_and_one_row_frames(m3s, H, W, r):
    """Frames two pixels wide or tall: staged windows and refine regions one
    column or one row wide (the staging's row/column split divides by 1)."""
    check(m3s, _pair(H, W, 7 * H + W), "%dx%d r%d" % (H, W, r), r=r)
    check(m3s, synth.identity_pair(H, W, 12), "identity %dx%d r%d" % (H, W, r), r=r)


@pytest.mark.parametrize("K,r", [(0, 3), (1, 3), (3, 0), (10, 1), (15, 8), (30, 2)])
def test_iterations_and_radius(m3s, K, r):
    check(m3s, _pair(48, 64, 7), "K%d r%d" % (K, r), K=K, r=r)


def test_p_init(m3s):
    """Tracking-style initialisation from given pixels (Sec. 3.2)."""
    pair = _pair(96, 128, 8)
    rng = np.random.Generator(np.random.PCG64(1))
    p_init = pair.proj + rng.normal(0, 1.5, size=pair.proj.shape)
    check(m3s, pair, "p_init", p_init=p_init, K=5)


def test_gates(m3s):
    """Distance gate on, angle gate off and a stricter confidence gate."""
    pair = _pair(96, 128, 9)
    check(m3s, pair, "dist gate", max_dist=0.2)
    # Without the angle gate, matches beyond the border are valid; their p* is
    # the fixed point of a non-zero residual, so p* is compared at residual
    # angles up to 1e-4 rad only (validity and idx are compared everywhere).
    check(m3s, pair, "no angle gate", max_theta=math.inf, p_theta_max=1e-4)
    check(m3s, pair, "conf 3", conf_min=3.0)


def test_bad_inputs(m3s):
    """Non-finite and zero points, bad reference pixels, non-finite p_init."""
    pair = _pair(48, 64, 10)
    pair = synth.Pair(pair.H, pair.W, pair.Xii.copy(), pair.Xji.copy(), pair.Dii, pair.Dji, pair.Qii, pair.Qji,
                      proj=pair.proj)
    pair.Xji[0, 0] = [np.nan, 1, 1]
    pair.Xji[1, 5] = [0, 0, 0]
    pair.Xji[2, 7] = [np.inf, 0, 1]
    pair.Xii[20, 30] = [np.nan, 0, 0]
    pair.Xii[21, 31] = [0, 0, 0]
    p_init = np.stack(synth.pixel_grid(48, 64), -1)
    p_init[3, 3] = [np.nan, 2]
    g, o, st = check(m3s, pair, "bad inputs", p_init=p_init)
    for y, x in [(0, 0), (1, 5), (2, 7), (3, 3)]:
        assert g["idx"][y, x] == -1 and not g["valid"][y, x] and g["theta"][y, x] == np.inf


@pytest.mark.parametrize("H,W", [(48, 64), (2, 2), (3, 7)])
def test_identity(m3s, H, W):
    p = synth.identity_pair(H, W, 12)
    g = run(m3s, p)
    xs, ys = synth.pixel_grid(H, W)
    assert np.abs(g["p"][..., 0] - xs).max() <= 1e-4 and np.abs(g["p"][..., 1] - ys).max() <= 1e-4
    assert (g["idx"] == np.arange(H * W).reshape(H, W)).all()
    assert g["valid"].all()
    check(m3s, p, "identity %dx%d" % (H, W))


def test_generic_descriptor_paths(m3s):
    """D != 24 and misaligned descriptors take the generic path; it must give the
    same bits as the register path for D = 24."""
    import torch
    pair = _pair(48, 64, 13, conf=False)
    check(m3s, synth.make_pair(48, 64, 14, D=7), "D7")
    check(m3s, synth.make_pair(48, 64, 15, D=64), "D64")
    t = parity.pair_tensors(pair)
    ref = parity.result_numpy(m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"]))
    N = 48 * 64 * 24
    bi = torch.empty(N + 1, device="cuda")[1:]
    bj = torch.empty(N + 1, device="cuda")[1:]
    bi.copy_(t["Dii"].reshape(-1))
    bj.copy_(t["Dji"].reshape(-1))
    assert bi.data_ptr() % 16 != 0
    mis = parity.result_numpy(m3s.match(t["Xii"], t["Xji"], bi.view(48, 64, 24), bj.view(48, 64, 24)))
    for k in ("p", "idx", "valid", "theta"):
        assert np.array_equal(ref[k], mis[k]), k


def test_tile_configs_bitwise_and_deterministic(m3s):
    """Every tile shape (global-memory and LDS refine) and repeated runs give identical bits."""
    pair = _pair(200, 264, 16)
    outs = []
    try:
        for tc in (0, 1, 2, 3, 4, 5, 6, 3):
            m3s.set_launch(tile_config=tc)
            outs.append(run(m3s, pair))
        m3s.set_launch(tile_config=5, xcd_remap=0)
        outs.append(run(m3s, pair))
    finally:
        m3s.set_launch()
    for o in outs[1:]:
        for k in ("p", "idx", "valid", "theta", "xhat"):
            assert np.array_equal(outs[0][k], o[k], equal_nan=True), k


def _run_cfg(m3s, pair, cfg, **prm):
    m3s.set_launch(tile_config=int(cfg))
    try:
        return run(m3s, pair, **prm)
    finally:
        m3s.set_launch()


def _with_desc(pair, Dii, Dji):
    return synth.Pair(pair.H, pair.W, pair.Xii, pair.Xji, np.ascontiguousarray(Dii, np.float32),
                      np.ascontiguousarray(Dji, np.float32), pair.Qii, pair.Qji, K=pair.K, r=pair.r, proj=pair.proj)


@pytest.mark.parametrize("case", ["near_ties", "exact_ties", "huge", "tiny", "nan_ref", "unnormalised",
                                  "ref_x200", "ref_x1000", "query_x300", "r4", "r5", "r6"])
def test_fp16_prefilter_is_exact(m3s, case):
    """The fp16 pre-filtered refine (tile configuration 5) returns the same bits
    as the exact global-memory scan (configuration 0) on adversarial descriptors:
    near-ties within the fp16 error, exact ties, magnitudes outside fp16, values
    in the fp16 subnormal range, NaN in the reference region, non-unit norms,
    reference magnitudes on either side of the scaled fp16 range (x200 stays in
    the pre-filter, x1000 sends its regions to the exact scan), query
    descriptors beyond it (per-query exact scan inside a pre-filtered tile), and
    radii that need two candidate masks or fall back to the exact scan."""
    base = _pair(96, 128, 17)
    rng = np.random.Generator(np.random.PCG64(zlib.crc32(case.encode())))
    Dii, Dji = base.Dii.astype(np.float64), base.Dji.astype(np.float64)
    prm = {}
    if case == "near_ties":
        Dii = Dii[..., :1].repeat(24, -1) * 0 + 1.0 / np.sqrt(24)
        Dii = Dii + rng.normal(0, 2e-5, Dii.shape)
        Dji = np.full_like(Dji, 1.0 / np.sqrt(24))
    elif case == "exact_ties":
        Dii = np.round(Dii * 4) / 4
        Dji = np.round(Dji * 4) / 4
    elif case == "huge":
        Dii = Dii * 1e5
    elif case == "tiny":
        Dii = Dii * 3e-6
        Dji = Dji * 7e-6
    elif case == "nan_ref":
        Dii = Dii.copy()
        Dii[40:43, 60:63, 5] = np.nan
    elif case == "unnormalised":
        Dii = Dii * rng.uniform(0.1, 30.0, Dii.shape[:2])[..., None]
        Dji = Dji * rng.uniform(0.1, 30.0, Dji.shape[:2])[..., None]
    elif case == "ref_x200":
        Dii = Dii * 200.0
    elif case == "ref_x1000":
        Dii = Dii * 1000.0
    elif case == "query_x300":
        Dji = Dji * 300.0
    elif case in ("r4", "r5", "r6"):
        prm["refine_radius"] = int(case[1])
    pair = _with_desc(base, Dii, Dji)
    a = _run_cfg(m3s, pair, "0", **prm)
    b = _run_cfg(m3s, pair, "5", **prm)
    c = _run_cfg(m3s, pair, "3", **prm)
    d = _run_cfg(m3s, pair, "6", **prm)
    for k in ("p", "idx", "valid", "theta"):
        assert np.array_equal(a[k], b[k], equal_nan=True), "%s: %s (fp16 pre-filter)" % (case, k)
        assert np.array_equal(a[k], c[k], equal_nan=True), "%s: %s (fp32 LDS)" % (case, k)
        assert np.array_equal(a[k], d[k], equal_nan=True), "%s: %s (fp16 pre-filter, 8x8 tiles)" % (case, k)


@pytest.mark.parametrize("levels", [2, 3])
def test_refine_levels(m3s, levels):
    """Coarse-to-fine refine (Sec. 3.2) vs the oracle on the 512x384 workload,
    and on position-code descriptors whose targets lie up to r(2^L - 1) px away;
    every tile configuration gives the same bits."""
    pair = synth.config_pair(2)
    check(m3s, pair, "levels %d" % levels, levels=levels)
    sys_path_pins()
    import pins
    base = _pair(96, 128, 21, conf=False)
    o0 = ora(base)
    m0 = np.floor(o0["p"] + 0.5).astype(int)
    xs, ys = synth.pixel_grid(base.H, base.W)
    rng = np.random.Generator(np.random.PCG64(40 + levels))
    reach = 3 * (2 ** levels - 1) - 1
    off = rng.integers(-reach, reach + 1, size=(base.H, base.W, 2))
    code = _with_desc(base, pins._position_code(xs, ys), pins._position_code(m0[..., 0] + off[..., 0], m0[..., 1] + off[..., 1]))
    g, o, st = check(m3s, code, "position code L%d" % levels, levels=levels)
    outs = [_run_cfg(m3s, code, c, refine_levels=levels) for c in ("0", "3", "5", "6")]
    for k in ("p", "idx", "valid", "theta"):
        assert all(np.array_equal(outs[0][k], o[k]) for o in outs[1:]), k


@pytest.mark.parametrize("levels", [2, 3, 4])
def test_refine_levels_fast_path(m3s, levels):
    """Coarse-to-fine in the fp16 tile configuration at 512x384, from
    previous-frame initial pixels (the tracking setting, Sec. 3.2): every level
    of every tile runs on the pre-filtered path, the levels whose regions exceed
    LDS (L = 3: the coarsest, L = 4: the coarsest two) staged in bands of rows,
    and the result equals the global-memory configuration bit for bit and the
    oracle."""
    pair = synth.config_pair(2)
    rng = np.random.Generator(np.random.PCG64(60 + levels))
    p_init = (pair.proj + rng.normal(0, 1.5, size=pair.proj.shape)).astype(np.float32)
    t = parity.pair_tensors(pair)
    outs, cnts = [], []
    for cfg in (5, 0):
        m3s.path_counters(reset=True)
        m3s.set_launch(tile_config=cfg)
        try:
            res = m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], parity.to_dev(p_init),
                            m3s.params(refine_levels=levels), want_xhat=True)
            outs.append(parity.result_numpy(res))
        finally:
            m3s.set_launch()
        cnts.append(m3s.path_counters(reset=True))
    print("levels", levels, "counters (fp16, global):", cnts)
    tiles = (384 // 16) * (512 // 16)
    assert cnts[0]["refine_global"] == 0
    if levels == 2:
        assert cnts[0]["refine_bands"] == 0
    else:
        # The coarsest level of most tiles is banded (near the image border the
        # clipped region fits LDS whole).
        assert 0.8 * tiles <= cnts[0]["refine_bands"] <= (levels - 2) * tiles
    for k in ("p", "idx", "valid", "theta", "xhat"):
        assert np.array_equal(outs[0][k], outs[1][k], equal_nan=True), k
    o = ora(pair, p_init.astype(np.float64), levels=levels)
    print(parity.compare(outs[0], o, "tracking L%d" % levels))


def sys_path_pins():
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    if here not in sys.path:
        sys.path.insert(0, here)


@pytest.mark.parametrize("H,W,frac", [(48, 64, 0.7), (384, 512, 0.9), (7, 5, 1.0), (33, 65, 0.0)])
def test_match_stats(m3s, H, W, frac):
    """Keyframe statistics on seeded idx / valid arrays (duplicates, -1 entries,
    all-invalid) equal the oracle's counts exactly."""
    import torch
    rng = np.random.Generator(np.random.PCG64(H * W))
    N = H * W
    idx = rng.integers(0, N, size=N).astype(np.int32)
    idx[rng.uniform(size=N) < 0.05] = -1
    idx[: N // 3] = idx[N // 3: 2 * (N // 3)]          # duplicates
    valid = (rng.uniform(size=N) < frac) & (idx >= 0)
    res = m3s.MatchResult(torch.zeros((H, W, 2), device="cuda"), torch.from_numpy(idx.reshape(H, W)).cuda(),
                          torch.from_numpy(valid.reshape(H, W).astype(np.uint8)).cuda(), None, None)
    got = m3s.match_stats(res).cpu().numpy().tolist()
    assert got == list(oracle.match_stats(idx, valid)), (got, oracle.match_stats(idx, valid))
    # End to end on a real match set: within the valid-flag disagreement.
    pair = _pair(48, 64, 7)
    t = parity.pair_tensors(pair)
    r = m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"])
    gs = m3s.match_stats(r).cpu().numpy()
    os_ = oracle.match_stats(*[ora(pair)[k] for k in ("idx", "valid")])
    assert abs(int(gs[0]) - os_[0]) <= 0.001 * 48 * 64 + 1 and abs(int(gs[1]) - os_[1]) <= 0.001 * 48 * 64 + 1
