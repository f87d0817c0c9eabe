"""Batched persistent launch: bitwise equal to per-pair launches, graph replays
equal to eager runs, and oracle parity on sampled edges at full size."""
import functools

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


def edge_inputs(m3s, pairs):
    out = []
    for p in pairs:
        t = parity.pair_tensors(p)
        out.append(m3s.EdgeInput(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], None, p.K, p.r))
    return out


def per_pair(m3s, edges):
    res = []
    for e in edges:
        prm = m3s.params(max_iter=e.max_iter, refine_radius=e.refine_radius)
        res.append(parity.result_numpy(m3s.match(e.Xii, e.Xji, e.Dii, e.Dji, e.Qii, e.Qji, None, prm,
                                                 want_xhat=True)))
    return res


def assert_same(a, b, label):
    for k in ("p", "idx", "valid", "theta", "xhat"):
        assert np.array_equal(a[k], b[k], equal_nan=True), "%s: %s differs" % (label, k)


@functools.lru_cache(maxsize=None)
def mixed_pairs():
    dims = [(48, 64, 10, 3), (37, 53, 5, 2), (96, 128, 15, 4), (2, 2, 7, 1), (64, 48, 12, 0), (130, 70, 8, 3)]
    return [synth.make_pair(H, W, 700 + k, K=K, r=r, conf=(k % 2 == 0)) for k, (H, W, K, r) in enumerate(dims)]


@pytest.mark.parametrize("graph,autotune", [(False, False), (True, False), (True, True), (False, True)])
def test_batched_equals_per_pair(m3s, graph, autotune):
    import torch
    edges = edge_inputs(m3s, mixed_pairs())
    ref = per_pair(m3s, edges)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = m3s.match_batched(edges, graph=graph, autotune=autotune, want_xhat=True)
    s.synchronize()
    for k, (a, b) in enumerate(zip(ref, outs)):
        assert_same(a, parity.result_numpy(b), "edge %d" % k)


def test_back_to_back_calls_without_synchronisation(m3s):
    """Twelve batched forwards, then twelve batched backwards, issued on one
    stream without a host synchronisation and alternating three edge sets
    (eager and graph submission): every call's edge table goes through a ring
    of eight pinned staging slots, so slots are reused while earlier calls may
    still be queued. Every call's outputs equal the per-pair launches (the
    forward bit for bit; the backward's dL/dX^j_i bit for bit and dL/dX^i_i
    up to the order of the fp32 atomics)."""
    import torch
    pairs = mixed_pairs()
    sets = [pairs[:3], pairs[3:], pairs[1:5]]
    edges = [edge_inputs(m3s, ps) for ps in sets]
    refs = [per_pair(m3s, e) for e in edges]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    outs = []
    print("case back-to-back batched forwards", flush=True)
    with torch.cuda.stream(s):
        for k in range(12):
            j = k % 3
            outs.append((j, m3s.match_batched(edges[j], graph=(k % 4 < 2), want_xhat=True, stream=s)))
    s.synchronize()
    for k, (j, o) in enumerate(outs):
        for e, (a, b) in enumerate(zip(refs[j], o)):
            assert_same(a, parity.result_numpy(b), "call %d edge %d" % (k, e))
    # Backward over the same edges from the per-pair matches.
    bins, brefs = [], []
    for j, es in enumerate(edges):
        bj, rj = [], []
        for e, r in zip(es, refs[j]):
            H, W = e.Xii.shape[:2]
            rng = np.random.Generator(np.random.PCG64(40 + H + W))
            p = parity.to_dev(r["p"])
            v = torch.from_numpy(r["valid"].astype(np.uint8)).cuda()
            gp = parity.to_dev(rng.normal(size=(H, W, 2)))
            gx = parity.to_dev(rng.normal(size=(H, W, 3)))
            bj.append(m3s.BwdEdgeInput(e.Xii, e.Xji, p, v, gp, gx))
            rj.append(m3s.match_backward(e.Xii, e.Xji, p, v, gp, gx))
        bins.append(bj)
        brefs.append(rj)
    torch.cuda.synchronize()
    bouts = []
    print("case back-to-back batched backwards", flush=True)
    with torch.cuda.stream(s):
        for k in range(12):
            j = k % 3
            bouts.append((j, m3s.match_backward_batched(bins[j], graph=(k % 4 < 2), stream=s)))
    s.synchronize()
    for k, (j, o) in enumerate(bouts):
        for e, ((ri, rj), (gi, gj)) in enumerate(zip(brefs[j], o)):
            assert torch.equal(rj, gj), (k, e)
            scale = max(float(ri.abs().max()), 1e-30)
            assert float((gi - ri).abs().max()) <= 1e-6 * scale, (k, e)


def test_graph_replays_with_new_contents(m3s):
    """The same shapes with new inputs replay the cached graph; every replay,
    with eager work and synchronisation between them, equals the eager result."""
    import torch
    s = torch.cuda.Stream()
    for rep in range(3):
        pairs = [synth.make_pair(H, W, 900 + 10 * rep + k, K=K, r=r)
                 for k, (H, W, K, r) in enumerate([(48, 64, 10, 3), (40, 56, 6, 2), (33, 65, 12, 4)])]
        edges = edge_inputs(m3s, pairs)
        ref = per_pair(m3s, edges)
        with torch.cuda.stream(s):
            outs = m3s.match_batched(edges, graph=True, want_xhat=True)
        s.synchronize()
        torch.zeros(1000, device="cuda").sum().item()  # unrelated eager work
        for k, (a, b) in enumerate(zip(ref, outs)):
            assert_same(a, parity.result_numpy(b), "replay %d edge %d" % (rep, k))
    # A different edge count takes a new graph.
    edges = edge_inputs(m3s, mixed_pairs()[:2])
    ref = per_pair(m3s, edges)
    with torch.cuda.stream(s):
        outs = m3s.match_batched(edges, graph=True, want_xhat=True)
    s.synchronize()
    for k, (a, b) in enumerate(zip(ref, outs)):
        assert_same(a, parity.result_numpy(b), "recapture edge %d" % k)


def _full_batch_check(m3s, pairs, sample, label):
    import torch
    edges = edge_inputs(m3s, pairs)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = m3s.match_batched(edges, graph=True, autotune=True, want_xhat=True)
    s.synchronize()
    print(label, "launch shape (grid, tile):", m3s.last_batched_config())
    ref = per_pair(m3s, [edges[k] for k in sample])
    for j, k in enumerate(sample):
        g = parity.result_numpy(outs[k])
        assert_same(ref[j], g, "%s edge %d" % (label, k))
        p = pairs[k]
        o = oracle.match_fwd(p.Xii, p.Xji, p.Dii, p.Dji, p.Qii, p.Qji, K=p.K, r=p.r)
        print(parity.compare(g, o, "%s edge %d (%dx%d K%d r%d)" % (label, k, p.H, p.W, p.K, p.r), pair=p, r=p.r))


def test_batched_64_edges_512x384(m3s):
    """64 edges at 512x384 in one launch; oracle parity on 6 sampled edges."""
    pairs = synth.batched_uniform()
    _full_batch_check(m3s, pairs, [0, 9, 21, 38, 50, 63], "64x512x384")


def test_batched_96_uneven_edges(m3s):
    """40 edges at 512x384, 32 at 384x512, 24 at 512x288, K in 5..15, r in 2..4."""
    pairs = synth.batched_uneven()
    _full_batch_check(m3s, pairs, [0, 17, 39, 40, 55, 71, 72, 88, 95], "uneven")


def test_every_launch_candidate_gives_identical_bits(m3s):
    """Every launch the autotuner can pick (tile configuration x grid, and for
    the fp16 configuration ray-window margin x LM unroll) writes the same bits
    as the per-pair launch."""
    import torch
    edges = edge_inputs(m3s, mixed_pairs())
    ref = per_pair(m3s, edges)
    cands = [(t, 64, -1, -1) for t in (0, 1, 2, 3, 4, 6)] + [(5, g, m, u) for g in (32, 1024) for m in (1, 2, 3)
                                                             for u in (1, 2)]
    s = torch.cuda.Stream()
    for t, g, m, u in cands:
        print("case launch tile %d grid %d margin %d unroll %d" % (t, g, m, u), flush=True)
        m3s.set_launch(tile_config=t, grid=g, ray_margin=m, lm_unroll=u)
        try:
            with torch.cuda.stream(s):
                outs = m3s.match_batched(edges, graph=False, want_xhat=True)
            s.synchronize()
            used = m3s.last_batched_launch()
        finally:
            m3s.set_launch()
        assert used["tile_config"] == t
        if t == 5:
            assert (used["ray_margin"], used["lm_unroll"]) == (m, u)
        for k, (a, b) in enumerate(zip(ref, outs)):
            assert_same(a, parity.result_numpy(b), "tile %d margin %d unroll %d edge %d" % (t, m, u, k))


def test_autotune_cache_file_round_trip(m3s, tmp_path):
    """The tuner writes its result to the cache file; after the in-memory
    caches are dropped, the file's entry (edited to a distinctive launch) is
    used as is, with no new tuning, and the outputs keep their bits."""
    import json
    import torch
    lib = m3s.load_library()
    lib.m3s_clear_caches()          # earlier tests' results would be written to the file too
    path = tmp_path / "tune.json"
    m3s.set_tune_cache(str(path))
    try:
        edges = edge_inputs(m3s, mixed_pairs()[:3])
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            a = m3s.match_batched(edges, graph=False, autotune=True, want_xhat=True)
        s.synchronize()
        data = json.loads(path.read_text())
        assert data["format"] == "m3s-autotune" and data["version"] == 1
        keys = [k for k in data["entries"] if "cu|" in k]
        assert len(keys) == 1
        tuned = m3s.last_batched_launch()
        assert data["entries"][keys[0]] == [tuned["tile_config"], tuned["grid"], tuned["ray_margin"], tuned["lm_unroll"]]
        data["entries"][keys[0]] = [5, 7, 3, 2]
        path.write_text(json.dumps(data))
        lib.m3s_clear_caches()
        m3s.set_tune_cache(str(path))
        with torch.cuda.stream(s):
            b = m3s.match_batched(edges, graph=True, autotune=True, want_xhat=True)
        s.synchronize()
        assert m3s.last_batched_launch() == dict(tile_config=5, grid=7, ray_margin=3, lm_unroll=2)
        for k, (x, y) in enumerate(zip(a, b)):
            assert_same(parity.result_numpy(x), parity.result_numpy(y), "reloaded edge %d" % k)
    finally:
        m3s.set_tune_cache(None)
        lib.m3s_clear_caches()


@pytest.mark.parametrize("levels", [2, 3, 4])
def test_batched_coarse_to_fine_equals_per_pair(m3s, levels):
    """The persistent kernel's multi-level refine equals the per-pair launch bit
    for bit; at L = 3 the coarsest levels that exceed LDS are staged in bands."""
    import torch
    edges = edge_inputs(m3s, mixed_pairs())
    ref = []
    for e in edges:
        prm = m3s.params(max_iter=e.max_iter, refine_radius=e.refine_radius, refine_levels=levels)
        ref.append(parity.result_numpy(m3s.match(e.Xii, e.Xji, e.Dii, e.Dji, e.Qii, e.Qji, None, prm,
                                                 want_xhat=True)))
    s = torch.cuda.Stream()
    m3s.path_counters(reset=True)
    with torch.cuda.stream(s):
        outs = m3s.match_batched(edges, prm=m3s.params(refine_levels=levels), graph=True, want_xhat=True)
    s.synchronize()
    cnt = m3s.path_counters(reset=True)
    print("L%d batched path counters:" % levels, cnt)
    if levels >= 3:
        assert cnt["refine_bands"] > 0
    for k, (a, b) in enumerate(zip(ref, outs)):
        assert_same(a, parity.result_numpy(b), "L%d edge %d" % (levels, k))
