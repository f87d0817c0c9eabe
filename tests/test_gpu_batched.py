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
