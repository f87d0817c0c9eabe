"""Inputs that force every fallback branch of the forward and backward kernels,
with the device path counters showing that the branch ran and the oracle (or
the exact global-memory path) showing that its results are right.

  * LM ray window above its LDS cap: query pixels shuffled, so a tile's
    queries reach cells everywhere after one iteration;
  * refine region above its LDS cap: the same scattered pixels with K = 0, so
    the refine windows of a tile lie all over the image;
  * backward corner window above its LDS cap: p* scattered over the image;
  * the batched kernel in every tile configuration (the global-memory and
    fp32-LDS modes as well as the default fp16 one).
"""
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


def scattered(H, W, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.stack([rng.uniform(0, W - 1, (H, W)), rng.uniform(0, H - 1, (H, W))], -1).astype(np.float32)


def run_counted(m3s, pair, tile_config, p_init=None, **prm):
    t = parity.pair_tensors(pair)
    m3s.path_counters(reset=True)
    m3s.set_launch(tile_config=tile_config)
    try:
        res = m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], parity.to_dev(p_init),
                        m3s.params(**prm), want_xhat=True)
        g = parity.result_numpy(res)
    finally:
        m3s.set_launch()
    return g, m3s.path_counters(reset=True)


def permuted_queries(pair, seed):
    """The pair with its query pixels shuffled: neighbouring queries then match
    pixels anywhere in the image (the method matches each query on its own)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(pair.H * pair.W)
    f = lambda a: None if a is None else np.ascontiguousarray(a.reshape(pair.H * pair.W, -1)[perm].reshape(a.shape))
    return synth.Pair(pair.H, pair.W, pair.Xii, f(pair.Xji), pair.Dii, f(pair.Dji), pair.Qii, f(pair.Qji),
                      K=pair.K, r=pair.r, proj=f(pair.proj))


@pytest.mark.parametrize("tile_config", [3, 5, 6])
def test_lm_window_overflow(m3s, tile_config):
    """Shuffled queries: after the first iteration a tile's queries sit on cells
    all over the image, so every tile's LM window exceeds the LDS cap and
    iterations 2..K read the ray records from global memory."""
    pair = permuted_queries(synth.make_pair(96, 128, 31), 5)
    print("case lm_window_overflow tile %d" % tile_config, flush=True)
    g, cnt = run_counted(m3s, pair, tile_config, None, max_iter=10)
    print(cnt)
    tiles = 48 if tile_config != 6 else 192   # 16 x 16 or 8 x 8 tiles
    assert cnt["lm_global"] >= 0.9 * tiles
    o = oracle.match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji, K=10, r=pair.r)
    print(parity.compare(g, o, "lm window overflow (tile %d)" % tile_config, pair=pair, r=pair.r))


@pytest.mark.parametrize("tile_config", [3, 5, 6])
def test_refine_region_overflow(m3s, tile_config):
    """K = 0 from scattered pixels: p* is the initial pixel, the tile's refine
    windows lie all over the image and the region exceeds LDS, so every tile
    scans global memory; with the angle gate off every match is valid and
    compared."""
    pair = synth.make_pair(96, 128, 32)
    pi = scattered(96, 128, 6)
    print("case refine_region_overflow tile %d" % tile_config, flush=True)
    g, cnt = run_counted(m3s, pair, tile_config, pi, max_iter=0, max_theta=float("inf"))
    print(cnt)
    assert cnt["refine_global"] == (48 if tile_config != 6 else 192)
    o = oracle.match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji, pi.astype(np.float64),
                         K=0, r=pair.r, max_theta=np.inf)
    st = parity.compare(g, o, "refine region overflow (tile %d)" % tile_config, p_theta_max=np.inf, pair=pair,
                        r=pair.r)
    print(st)
    assert st["idx_compared"] > 0.9 * pair.H * pair.W


def test_fp16_range_fallbacks_counted(m3s):
    """Reference descriptors beyond the scaled fp16 range send their tiles to the
    exact scan, oversized query descriptors their queries, r = 6 every tile; the
    bits equal the global-memory configuration's."""
    base = synth.make_pair(96, 128, 17)
    cases = [("ref_x1000", base.Dii * 1000.0, base.Dji, {}, "refine_global"),
             ("query_x300", base.Dii, base.Dji * 300.0, {}, "refine_query"),
             ("r6", base.Dii, base.Dji, {"refine_radius": 6}, "refine_global")]
    for name, Dii, Dji, prm, key in cases:
        pair = synth.Pair(base.H, base.W, base.Xii, base.Xji, np.ascontiguousarray(Dii, np.float32),
                          np.ascontiguousarray(Dji, np.float32), base.Qii, base.Qji, K=base.K, r=base.r,
                          proj=base.proj)
        print("case fp16 range %s" % name, flush=True)
        g5, c5 = run_counted(m3s, pair, 5, **prm)
        g0, c0 = run_counted(m3s, pair, 0, **prm)
        print(name, c5)
        assert c5[key] > 0, (name, c5)
        for k in ("p", "idx", "valid", "theta"):
            assert np.array_equal(g5[k], g0[k], equal_nan=True), (name, k)


def test_bwd_window_overflow(m3s):
    """p* scattered over the image: every backward tile's corner window exceeds
    the LDS accumulator, so its gradients go to dL/dX^i_i by direct global
    atomics; both outputs agree with the oracle's adjoint element by element."""
    import torch
    H, W = 96, 128
    pair = synth.make_pair(H, W, 33)
    p = scattered(H, W, 7)
    valid = np.ones((H, W), bool)
    rng = np.random.Generator(np.random.PCG64(8))
    gp = rng.normal(size=(H, W, 2)).astype(np.float32)
    gx = rng.normal(size=(H, W, 3)).astype(np.float32)
    print("case bwd_window_overflow", flush=True)
    m3s.path_counters(reset=True)
    gi, gj = m3s.match_backward(parity.to_dev(pair.Xii), parity.to_dev(pair.Xji), parity.to_dev(p),
                                torch.from_numpy(valid.astype(np.uint8)).cuda(), parity.to_dev(gp),
                                parity.to_dev(gx))
    torch.cuda.synchronize()
    cnt = m3s.path_counters(reset=True)
    print(cnt)
    assert cnt["bwd_direct"] == 48
    oi, oj = oracle.match_bwd(pair.Xii, pair.Xji, p.astype(np.float64), valid, gp, gx)
    gi, gj = gi.cpu().numpy(), gj.cpu().numpy()
    ei = np.abs(gi - oi).max() / np.abs(oi).max()
    ej = np.abs(gj - oj).max() / np.abs(oj).max()
    print(dict(max_rel_dXii=float(ei), max_rel_dXji=float(ej)))
    assert ei <= 1e-4 and ej <= 1e-4


def _edges(m3s, pairs):
    out = []
    for p in pairs:
        t = parity.pair_tensors(p)
        out.append(m3s.EdgeInput(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], None, p.K, p.r))
    return out


@pytest.mark.parametrize("tile_config", [0, 1, 2, 3, 4, 5, 6])
def test_batched_every_tile_config(m3s, tile_config):
    """The persistent kernel in each tile configuration equals the per-pair
    launch bit for bit, and two edges agree with the oracle."""
    import torch
    dims = [(48, 64, 10, 3), (37, 53, 5, 2), (96, 128, 15, 4), (64, 48, 12, 0), (130, 70, 8, 3)]
    pairs = [synth.make_pair(H, W, 1700 + k, K=K, r=r, conf=(k % 2 == 0)) for k, (H, W, K, r) in enumerate(dims)]
    edges = _edges(m3s, pairs)
    ref = []
    for e in edges:
        prm = m3s.params(max_iter=e.max_iter, refine_radius=e.refine_radius)
        ref.append(parity.result_numpy(m3s.match(e.Xii, e.Xji, e.Dii, e.Dji, e.Qii, e.Qji, None, prm,
                                                 want_xhat=True)))
    print("case batched tile %d" % tile_config, flush=True)
    m3s.set_launch(tile_config=tile_config, grid=64)
    try:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            outs = m3s.match_batched(edges, graph=False, want_xhat=True)
        s.synchronize()
        assert m3s.last_batched_config() == (64, tile_config)
    finally:
        m3s.set_launch()
    for k, (a, b) in enumerate(zip(ref, outs)):
        b = parity.result_numpy(b)
        for key in ("p", "idx", "valid", "theta", "xhat"):
            assert np.array_equal(a[key], b[key], equal_nan=True), (k, key)
    for k in (0, 2):
        p = pairs[k]
        o = oracle.match_fwd(p.Xii, p.Xji, p.Dii, p.Dji, p.Qii, p.Qji, K=p.K, r=p.r)
        print(parity.compare(parity.result_numpy(outs[k]), o, "tile %d edge %d" % (tile_config, k), pair=p, r=p.r))


def test_banded_level_fallbacks(m3s):
    """Coarse to fine at L = 3 from previous-frame pixels: the coarsest level's
    regions exceed LDS and are staged and pre-filtered in bands of rows.
    Reference descriptors beyond the scaled fp16 range in the lower rows make
    some of those levels fail the range test in a later band (exact global
    scan of that level instead), and oversized query descriptors send their
    queries to the exact scan from the first band.  The bits equal the
    global-memory configuration's, and the plain case agrees with the oracle."""
    base = synth.make_pair(96, 128, 41)
    rng = np.random.Generator(np.random.PCG64(41))
    p_init = (base.proj + rng.normal(0, 1.5, size=base.proj.shape)).astype(np.float32)
    big_ref = base.Dii.copy()
    big_ref[64:] *= 1000.0
    big_query = base.Dji.copy()
    big_query[10:12, 40:60] *= 300.0
    cases = [("plain", base.Dii, base.Dji, ()), ("ref_rows_x1000", big_ref, base.Dji, ("refine_global",)),
             ("query_x300", base.Dii, big_query, ("refine_query",))]
    for name, Dii, Dji, keys in cases:
        pair = synth.Pair(base.H, base.W, base.Xii, base.Xji, np.ascontiguousarray(Dii, np.float32),
                          np.ascontiguousarray(Dji, np.float32), base.Qii, base.Qji, K=base.K, r=base.r,
                          proj=base.proj)
        print("case banded levels %s" % name, flush=True)
        g5, c5 = run_counted(m3s, pair, 5, p_init, refine_levels=3)
        g0, _ = run_counted(m3s, pair, 0, p_init, refine_levels=3)
        print(name, c5)
        assert c5["refine_bands"] > 0, (name, c5)
        for key in keys:
            assert c5[key] > 0, (name, key, c5)
        for k in ("p", "idx", "valid", "theta", "xhat"):
            assert np.array_equal(g5[k], g0[k], equal_nan=True), (name, k)
        if name == "plain":
            o = oracle.match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji,
                                 p_init.astype(np.float64), K=pair.K, r=pair.r, levels=3)
            print(parity.compare(g5, o, "banded levels", pair=pair, r=pair.r, levels=3))
