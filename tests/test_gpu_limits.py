"""The forward at the largest frame the library accepts (H * W = 2^26 pixels).

At any size an identity pair (X^j_i = X^i_i, D^j_i = D^i_i) returns every
pixel to itself: the LM starts on a zero residual up to the fp32 rounding of
the renormalised ray, so p* stays within 1e-3 px of the query's own pixel (the
parity bar: beyond x = 4096 one fp32 step of a coordinate is 4.9e-4 px, so a
rounding-level LM step moves p by that much) and theta below 1e-6, and the refine
selects the own pixel because generic random unit descriptors are uniquely
most similar to themselves.
The pair is generated on the device (about 20 GB of device memory); the
check runs there too.
"""
import pytest
import torch

from paper_2412_12392_amd import match, params

pytestmark = pytest.mark.gpu


def test_identity_at_max_pixels():
    H, W = 8192, 8192                      # M3S_MAX_PIXELS = 2^26
    d = "cuda:0"
    print("limits case identity", H, W, flush=True)
    g = torch.Generator(device=d).manual_seed(7)
    ys = torch.arange(H, device=d, dtype=torch.float32).view(H, 1).expand(H, W)
    xs = torch.arange(W, device=d, dtype=torch.float32).view(1, W).expand(H, W)
    f = max(H, W) / 2.0
    u, v = (xs - W / 2.0) / f, (ys - H / 2.0) / f
    z = 2.0 + 0.3 * torch.sin(3 * u) * torch.cos(2 * v) + 0.1 * u + 0.05 * v
    X = torch.stack([u * z, v * z, z], dim=-1).contiguous()
    del ys, xs, u, v, z
    D = torch.randn((H, W, 24), generator=g, device=d)
    D /= D.norm(dim=-1, keepdim=True)
    res = match(X, X, D, D, prm=params(max_iter=10, refine_radius=3))
    torch.cuda.synchronize()
    iy = torch.arange(H, device=d, dtype=torch.float32).view(H, 1)
    ix = torch.arange(W, device=d, dtype=torch.float32).view(1, W)
    assert float((res.p[..., 0] - ix).abs().max()) <= 1e-3
    assert float((res.p[..., 1] - iy).abs().max()) <= 1e-3
    own = (torch.arange(H, device=d).view(H, 1) * W + torch.arange(W, device=d).view(1, W)).to(torch.int32)
    assert torch.equal(res.idx, own)
    assert bool((res.valid == 1).all())
    assert float(res.theta.abs().max()) <= 1e-6
