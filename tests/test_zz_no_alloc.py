"""m3s_match_fwd_noalloc (static device scratch, no allocation) against
m3s_match_fwd (caller workspace) through the C ABI: identical bits on two calls
in a row, the second on a smaller pair, and a clear error above the limit."""
import numpy as np
import pytest

import parity
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m3s():
    import paper_2412_12392_amd as m
    m.load_library()
    return m


def _outs(m3s, H, W):
    import torch
    from paper_2412_12392_amd import binding
    return binding._alloc_outputs(H, W, torch.device("cuda"), True, True)


def test_noalloc_matches_workspace_entry_point(m3s):
    import torch
    for H, W, seed in [(384, 512, 7100), (37, 53, 7101)]:
        print("case noalloc %dx%d" % (H, W), flush=True)
        pair = synth.make_pair(H, W, seed)
        t = parity.pair_tensors(pair)
        ref = parity.result_numpy(m3s.match(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"],
                                            want_xhat=True))
        out = _outs(m3s, H, W)
        torch.cuda.synchronize()
        m3s.match_noalloc(t["Xii"], t["Xji"], t["Dii"], t["Dji"], t["Qii"], t["Qji"], out=out)
        got = parity.result_numpy(out)
        for k in ("p", "idx", "valid", "theta", "xhat"):
            assert np.array_equal(ref[k], got[k], equal_nan=True), (H, W, k)


def test_noalloc_rejects_oversized_pair(m3s):
    import torch
    from paper_2412_12392_amd import _lib
    H, W = 520, 512                     # 266,240 > 2^18 pixels
    X = torch.ones((H, W, 3), device="cuda")
    D = torch.ones((H, W, 24), device="cuda")
    out = _outs(m3s, H, W)
    with pytest.raises(m3s.M3SError) as e:
        m3s.match_noalloc(X, X, D, D, out=out)
    assert e.value.status == 2 and "M3S_NOALLOC_MAX_PIXELS" in str(e.value)
    assert _lib.M3S_NOALLOC_MAX_PIXELS == 1 << 18
