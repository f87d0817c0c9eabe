"""Helpers of the GPU parity tests: run libm3s and the oracle on the same seeded
inputs and compare them to the matching contract.

Contract (fp32 device path vs fp64 oracle):
  * continuous p* within 1e-3 px and residual angle within 1e-5 rad on the
    queries both sides call valid;
  * refined idx identical wherever both are valid, the oracle's top-two window
    scores differ by more than 1e-5 and the oracle's p* is at least 1e-3 px
    away from a rounding boundary (x.5) in both axes, so that both sides
    search the same window (an fp32 dot product of unit 24-dim descriptors is
    within 24 * 2^-24 < 1.5e-6 of the exact value, so a gap above 1e-5 orders
    the two best candidates the same way on both sides);
  * valid flags agree on >= 99.9 % of queries.
"""
from __future__ import annotations

import numpy as np

P_TOL = 1e-3
THETA_TOL = 1e-5
GAP_MIN = 1e-5
STRADDLE = 1e-3
VALID_AGREE = 0.999


def to_dev(a, device="cuda"):
    import torch
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)


def pair_tensors(pair, device="cuda"):
    return dict(Xii=to_dev(pair.Xii, device), Xji=to_dev(pair.Xji, device), Dii=to_dev(pair.Dii, device),
                Dji=to_dev(pair.Dji, device), Qii=to_dev(pair.Qii, device), Qji=to_dev(pair.Qji, device))


def result_numpy(res):
    import torch
    torch.cuda.synchronize()
    out = dict(p=res.p.cpu().numpy().astype(np.float64), idx=res.idx.cpu().numpy(),
               valid=res.valid.cpu().numpy().astype(bool))
    if res.theta is not None:
        out["theta"] = res.theta.cpu().numpy().astype(np.float64)
    if res.xhat is not None:
        out["xhat"] = res.xhat.cpu().numpy().astype(np.float64)
    return out


def compare(gpu: dict, ora: dict, label: str = "", strict: bool = True, p_theta_max: float | None = None) -> dict:
    """Compare one pair's outputs; returns the statistics (asserts if strict).

    p_theta_max: compare p* and theta only where the oracle's residual angle is
    at most this (for runs with the angle gate off, where matches beyond the
    image border are valid but their p* is not a zero-residual root).
    """
    vg, vo = gpu["valid"], ora["valid"]
    both = vg & vo
    n = vg.size
    agree = float((vg == vo).mean())
    st = dict(label=label, queries=int(n), valid_oracle=int(vo.sum()), valid_gpu=int(vg.sum()),
              valid_both=int(both.sum()), valid_agreement=agree)
    cont = both if p_theta_max is None else both & (ora["theta"] <= p_theta_max)
    if p_theta_max is not None:
        st["p_compared"] = int(cont.sum())
    if cont.any():
        dp = np.abs(gpu["p"] - ora["p"]).max(-1)[cont]
        st["max_dp_px"] = float(dp.max())
        if "theta" in gpu:
            st["max_dtheta"] = float(np.abs(gpu["theta"][cont] - ora["theta"][cont]).max())
    else:
        st.update(max_dp_px=0.0, max_dtheta=0.0)
    if both.any():
        frac = ora["p"] - np.floor(ora["p"])
        straddle = (np.abs(frac - 0.5) < STRADDLE).any(-1)
        comparable = both & (ora["gap"] > GAP_MIN) & ~straddle
        st["idx_compared"] = int(comparable.sum())
        st["idx_excluded_gap"] = int((both & ~(ora["gap"] > GAP_MIN)).sum())
        st["idx_excluded_straddle"] = int((both & straddle).sum())
        st["idx_mismatch"] = int((gpu["idx"] != ora["idx"])[comparable].sum())
    else:
        st.update(idx_compared=0, idx_mismatch=0)
    # Queries the oracle rejects as bad input must be rejected the same way.
    bad = ora["idx"] == -1
    st["bad_input_mismatch"] = int(((gpu["idx"] != -1) | vg)[bad].sum())
    if strict:
        assert st["max_dp_px"] <= P_TOL, st
        assert st.get("max_dtheta", 0.0) <= THETA_TOL, st
        assert st["idx_mismatch"] == 0, st
        assert agree >= VALID_AGREE, st
        assert st["bad_input_mismatch"] == 0, st
    return st
