"""GPU backward (implicit adjoint) against the FP64 oracle's adjoint, and the
autograd.Function end to end."""
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


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _fed(m3s, pair, seed):
    """Oracle p* and mask fed to both backward implementations (same inputs)."""
    import torch
    o = oracle.match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji, K=20, r=pair.r)
    p32 = o["p"].astype(np.float32)
    rng = np.random.Generator(np.random.PCG64(seed))
    gp = rng.normal(size=p32.shape).astype(np.float32)
    gx = rng.normal(size=pair.Xii.shape).astype(np.float32)
    gi, gj = m3s.match_backward(parity.to_dev(pair.Xii), parity.to_dev(pair.Xji), parity.to_dev(p32),
                                torch.from_numpy(o["valid"].astype(np.uint8)).cuda(), parity.to_dev(gp),
                                parity.to_dev(gx))
    torch.cuda.synchronize()
    oi, oj = oracle.match_bwd(pair.Xii, pair.Xji, p32.astype(np.float64), o["valid"], gp, gx)
    return gi.cpu().numpy(), gj.cpu().numpy(), oi, oj, o


@pytest.mark.parametrize("H,W,seed", [(48, 64, 501), (384, 512, 502), (37, 53, 503)])
def test_bwd_matches_oracle_adjoint(m3s, H, W, seed):
    pair = synth.make_pair(H, W, seed)
    gi, gj, oi, oj, o = _fed(m3s, pair, seed)
    ei, ej = rel_l2(gi, oi), rel_l2(gj, oj)
    mi = float(np.abs(gi - oi).max() / np.abs(oi).max())
    mj = float(np.abs(gj - oj).max() / np.abs(oj).max())
    print(dict(shape=(H, W), rel_l2_dXii=ei, rel_l2_dXji=ej, max_rel_dXii=mi, max_rel_dXji=mj))
    assert ei <= 1e-4 and ej <= 1e-4
    # Element by element, both outputs within 1e-4 of their largest entry
    # (same p* and mask on both sides, so every pixel is compared).
    assert mi <= 1e-4 and mj <= 1e-4
    assert (gj[~o["valid"]] == 0).all()


@pytest.mark.parametrize("scale", [1e-30, 1e-12, 1.0, 1e12, 1e30])
def test_bwd_gradient_scales(m3s, scale):
    """The LDS window sums fixed-point numbers scaled per tile from the tile's
    largest |g|: incoming gradients from 1e-30 to 1e30 (with a 1e-6 .. 1
    spread inside the image, so the smallest reach fp32 subnormals at 1e-30)
    give dL/dX^i_i within 1e-4 of its largest entry, element by element,
    against the oracle's adjoint on the same p* and mask."""
    import torch
    pair = synth.make_pair(48, 64, 506)
    o = oracle.match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji, K=20, r=pair.r)
    p32 = o["p"].astype(np.float32)
    rng = np.random.Generator(np.random.PCG64(507))
    spread = 10.0 ** rng.uniform(-6, 0, size=(pair.H, pair.W, 1))
    gp = (rng.normal(size=p32.shape) * spread * scale).astype(np.float32)
    gx = (rng.normal(size=pair.Xii.shape) * spread * scale).astype(np.float32)
    print("case bwd scale %g" % scale, flush=True)
    gi, gj = m3s.match_backward(parity.to_dev(pair.Xii), parity.to_dev(pair.Xji), parity.to_dev(p32),
                                torch.from_numpy(o["valid"].astype(np.uint8)).cuda(), parity.to_dev(gp),
                                parity.to_dev(gx))
    torch.cuda.synchronize()
    oi, oj = oracle.match_bwd(pair.Xii, pair.Xji, p32.astype(np.float64), o["valid"], gp.astype(np.float64),
                              gx.astype(np.float64))
    gi, gj = gi.cpu().numpy(), gj.cpu().numpy()
    assert np.isfinite(gi).all() and np.isfinite(gj).all()
    mi = float(np.abs(gi - oi).max() / np.abs(oi).max())
    mj = float(np.abs(gj - oj).max() / np.abs(oj).max())
    print(dict(scale=scale, max_rel_dXii=mi, max_rel_dXji=mj))
    assert mi <= 1e-4 and mj <= 1e-4


def test_bwd_deterministic_query_side(m3s):
    pair = synth.make_pair(96, 128, 504)
    a = _fed(m3s, pair, 1)
    b = _fed(m3s, pair, 1)
    assert np.array_equal(a[1], b[1])
    assert rel_l2(a[0], b[0]) <= 1e-6


def test_autograd_function_end_to_end(m3s):
    """L = sum over valid matches of |xhat - x|^2 through MatchFunction; the
    gradient equals the oracle's implicit adjoint plus the direct term, on the
    same forward matches."""
    import torch
    pair = synth.make_pair(48, 64, 505, conf=False)
    Xi = parity.to_dev(pair.Xii).requires_grad_(True)
    Xj = parity.to_dev(pair.Xji).requires_grad_(True)
    p, xhat, idx, valid, theta = m3s.MatchFunction.apply(Xi, Xj, parity.to_dev(pair.Dii), parity.to_dev(pair.Dji),
                                                         None, None, None, m3s.params(max_iter=20))
    m = valid.bool()
    L = ((xhat - Xj) ** 2).sum(-1)[m].sum()
    L.backward()
    torch.cuda.synchronize()
    pg = p.detach().cpu().numpy().astype(np.float64)
    vg = valid.cpu().numpy().astype(bool)
    xh = xhat.detach().cpu().numpy().astype(np.float64)
    gx = 2.0 * (xh - pair.Xji) * vg[..., None]
    oi, oj = oracle.match_bwd(pair.Xii, pair.Xji, pg, vg, None, gx)
    oj = oj - gx
    ei = rel_l2(Xi.grad.cpu().numpy(), oi)
    ej = rel_l2(Xj.grad.cpu().numpy(), oj)
    print(dict(rel_l2_dXii=ei, rel_l2_dXji=ej))
    assert ei <= 1e-4 and ej <= 1e-4


def test_fwd_bwd_full_size_sampled(m3s):
    """512x384 fwd then bwd on the GPU's own matches vs the oracle's fwd + bwd:
    per-query gradients agree where both sides call the match valid."""
    import torch
    pair = synth.make_pair(384, 512, 5000)
    t = parity.pair_tensors(pair)
    res = m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], want_xhat=True)
    v = res.valid.bool()
    gx = (2.0 * (res.xhat - t["Xji"]) * v[..., None]).contiguous()
    gi, gj = m3s.match_backward(t["Xii"], t["Xji"], res.p, res.valid, torch.zeros_like(res.p), gx)
    torch.cuda.synchronize()
    o = oracle.match_fwd(pair.Xii, pair.Xji, pair.Dii, pair.Dji, pair.Qii, pair.Qji)
    ogx = 2.0 * (o["xhat"] - pair.Xji) * o["valid"][..., None]
    oi, oj = oracle.match_bwd(pair.Xii, pair.Xji, o["p"], o["valid"], None, ogx)
    vg = res.valid.cpu().numpy().astype(bool)
    both = o["valid"] & vg
    # The exact sampler derivative is one-sided at bilinear cell edges, so a
    # query whose p* lies within 1e-4 px of one may sit in different cells on
    # the two sides: its own dXji entry and the dXii entries of the corners it
    # touches on either side are left out, and so are the corners touched by
    # queries that only one side calls valid.
    frac = o["p"] - np.floor(o["p"])
    edge = ((frac < 1e-4) | (frac > 1 - 1e-4)).any(-1)
    skip = (both & edge) | (o["valid"] != vg)
    gp = res.p.cpu().numpy().astype(np.float64)
    touched = corner_pixels(o["p"], skip) | corner_pixels(gp, skip)
    print(dict(valid_both=int(both.sum()), cell_edge_excluded=int((both & edge).sum()),
               dXii_pixels_excluded=int(touched.sum())))
    both &= ~edge
    gj = gj.cpu().numpy()
    gi = gi.cpu().numpy()
    err = np.abs(gj - oj)[both].max() / np.abs(oj[both]).max()
    keep = ~touched
    err_i = np.abs(gi - oi)[keep].max() / np.abs(oi).max()
    print(dict(max_rel_dXji_valid_both=float(err), max_rel_dXii_compared=float(err_i), rel_l2_dXii=rel_l2(gi, oi)))
    assert err <= 1e-3
    assert err_i <= 1e-3


def corner_pixels(p, mask):
    """Pixels that are bilinear corners of p for the queries in mask."""
    H, W = mask.shape
    out = np.zeros((H, W), bool)
    q = p[mask]
    x0 = np.clip(np.minimum(np.floor(q[:, 0]).astype(int), W - 2), 0, W - 2)
    y0 = np.clip(np.minimum(np.floor(q[:, 1]).astype(int), H - 2), 0, H - 2)
    for dy in (0, 1):
        for dx in (0, 1):
            out[y0 + dy, x0 + dx] = True
    return out


def test_bwd_batched_matches_per_edge(m3s):
    """m3s_match_bwd_batched over edges of mixed size (with and without
    grad_xhat) against m3s_match_bwd per edge: dXji bit for bit, dXii up to the
    order of the fp32 atomics; eager, graph capture and graph replay; two edges
    against the oracle's adjoint element by element."""
    import torch
    dims = [(48, 64), (37, 53), (96, 128), (2, 2), (130, 70)]
    pairs = [synth.make_pair(H, W, 820 + k) for k, (H, W) in enumerate(dims)]
    inputs, refs, fed = [], [], []
    for k, pr in enumerate(pairs):
        t = parity.pair_tensors(pr)
        res = m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], want_xhat=True)
        rng = np.random.Generator(np.random.PCG64(900 + k))
        gp = parity.to_dev(rng.normal(size=(pr.H, pr.W, 2)))
        gx = None if k == 1 else parity.to_dev(rng.normal(size=(pr.H, pr.W, 3)))
        inputs.append(m3s.BwdEdgeInput(t["Xii"], t["Xji"], res.p, res.valid, gp, gx))
        refs.append(m3s.match_backward(t["Xii"], t["Xji"], res.p, res.valid, gp, gx))
        fed.append((res.p, res.valid, gp, gx))
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for rep, graph in enumerate((False, True, True)):
        print("case bwd batched rep %d graph %s" % (rep, graph), flush=True)
        with torch.cuda.stream(s):
            outs = m3s.match_backward_batched(inputs, graph=graph)
        s.synchronize()
        torch.zeros(100, device="cuda").sum().item()  # unrelated eager work between replays
        for k, ((ri, rj), (gi, gj)) in enumerate(zip(refs, outs)):
            assert torch.equal(rj, gj), (rep, k)
            scale = max(float(ri.abs().max()), 1e-30)
            assert float((gi - ri).abs().max()) <= 1e-6 * scale, (rep, k)
    for k in (0, 2):
        p, v, gp, gx = fed[k]
        oi, oj = oracle.match_bwd(pairs[k].Xii, pairs[k].Xji, p.cpu().numpy().astype(np.float64),
                                  v.cpu().numpy().astype(bool), gp.cpu().numpy(),
                                  None if gx is None else gx.cpu().numpy())
        gi, gj = (a.cpu().numpy() for a in outs[k])
        mi = float(np.abs(gi - oi).max() / np.abs(oi).max())
        mj = float(np.abs(gj - oj).max() / np.abs(oj).max())
        print(dict(edge=k, max_rel_dXii=mi, max_rel_dXji=mj))
        assert mi <= 1e-4 and mj <= 1e-4


def test_bwd_batched_accumulate(m3s):
    """M3S_BWD_ACCUMULATE: the batched backward adds its dL/dX^i_i to the
    buffers' contents (no zeroing launch) and still overwrites dL/dX^j_i.  Into
    zeroed buffers it equals the plain call up to the order of the fp32 atomics;
    into buffers holding G0 it gives G0 plus that; two edges sharing one
    dL/dX^i_i buffer (the same keyframe) sum their gradients; eager and graph."""
    import torch
    dims = [(48, 64), (37, 53), (96, 128)]
    pairs = [synth.make_pair(H, W, 840 + k) for k, (H, W) in enumerate(dims)]
    inputs = []
    for k, pr in enumerate(pairs):
        t = parity.pair_tensors(pr)
        res = m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], want_xhat=True)
        rng = np.random.Generator(np.random.PCG64(940 + k))
        gp = parity.to_dev(rng.normal(size=(pr.H, pr.W, 2)))
        gx = None if k == 1 else parity.to_dev(rng.normal(size=(pr.H, pr.W, 3)))
        inputs.append(m3s.BwdEdgeInput(t["Xii"], t["Xji"], res.p, res.valid, gp, gx))
    ref = m3s.match_backward_batched(inputs, graph=False)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for graph in (False, True, True):
        print("case bwd accumulate graph %s" % graph, flush=True)
        g0 = [parity.to_dev(np.random.Generator(np.random.PCG64(950 + k)).normal(size=(H, W, 3)))
              for k, (H, W) in enumerate(dims)]
        outs = [(g.clone(), torch.full_like(g, float("nan"))) for g in g0]
        with torch.cuda.stream(s):
            m3s.match_backward_batched(inputs, graph=graph, outs=outs, accumulate=True)
        s.synchronize()
        for k, ((ri, rj), (gi, gj)) in enumerate(zip(ref, outs)):
            assert torch.equal(rj, gj), k
            want = g0[k] + ri
            scale = max(float(want.abs().max()), 1e-30)
            assert float((gi - want).abs().max()) <= 2e-6 * scale, (graph, k)
        zeros = [(torch.zeros_like(ri), torch.empty_like(rj)) for ri, rj in ref]
        with torch.cuda.stream(s):
            m3s.match_backward_batched(inputs, graph=graph, outs=zeros, accumulate=True)
        s.synchronize()
        for k, ((ri, _), (gi, _)) in enumerate(zip(ref, zeros)):
            scale = max(float(ri.abs().max()), 1e-30)
            assert float((gi - ri).abs().max()) <= 1e-6 * scale, (graph, k)
    # Two edges of one keyframe into one dL/dX^i_i buffer.
    shared = torch.zeros_like(ref[0][0])
    two = [inputs[0], inputs[0]]
    with torch.cuda.stream(s):
        m3s.match_backward_batched(two, graph=False, outs=[(shared, torch.empty_like(shared)),
                                                           (shared, torch.empty_like(shared))], accumulate=True)
    s.synchronize()
    scale = max(float(ref[0][0].abs().max()), 1e-30)
    assert float((shared - 2.0 * ref[0][0]).abs().max()) <= 2e-6 * scale
