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

Beyond the contract, every query that is not rejected as bad input is checked
on its own terms (when the pair's descriptors are given, single-level refine):
  * p* and theta also agree on queries both sides converged (residual angle
    <= 1e-4 rad on both sides), whatever the gates decided, and theta agrees
    within 1e-5 rad on every good query, converged or not (beyond the image
    border theta is the angle to the nearest border ray, a minimum, and
    insensitive to where along the border p* stops);
  * its idx is a correct refine from the GPU's own window centre (p* rounded
    half up in fp32, as the kernel does): a candidate of that window whose
    exact (fp64) score is within the fp32 rounding of the two dot products
    (D * 2^-24 |q| |d| each) of the window's exact maximum.  Where the top-two
    gap exceeds those bounds this admits only the exact first maximum; at
    near-ties and for queries whose oracle p* straddles a rounding boundary
    (both excluded from the bit-exact comparison above) it checks that the
    GPU's choice is one of the correct answers.
"""
from __future__ import annotations

import numpy as np

P_TOL = 1e-3
THETA_TOL = 1e-5
GAP_MIN = 1e-5
STRADDLE = 1e-3
VALID_AGREE = 0.999
CONVERGED_THETA = 1e-4


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


def window_centre(p):
    """Refine window centre of the kernel: floor(p + 0.5) evaluated in fp32."""
    p32 = np.asarray(p, np.float32)
    return np.floor(p32 + np.float32(0.5)).astype(np.int64)


def idx_admissible(Dii, Dji, p, idx, r, mask, chunk=16384):
    """Per query of `mask`: True when idx is a correct single-level refine from
    the window centred on round-half-up(p) (see the module docstring), False
    when it is not, and None (excluded) when the window holds a non-finite
    score.  Returns (ok, checked, nonfinite) boolean arrays over the queries."""
    H, W, D = Dii.shape
    Di = Dii.reshape(-1, D).astype(np.float64)
    Dj = Dji.reshape(-1, D).astype(np.float64)
    dn = np.linalg.norm(Di, axis=1)
    qn = np.linalg.norm(Dj, axis=1)
    cen = window_centre(np.asarray(p).reshape(-1, 2))
    flat_idx = np.asarray(idx).reshape(-1).astype(np.int64)
    sel = np.flatnonzero(np.asarray(mask).reshape(-1))
    ok = np.zeros(H * W, bool)
    nonfin = np.zeros(H * W, bool)
    off = np.arange(-r, r + 1)
    dy, dx = np.meshgrid(off, off, indexing="ij")
    dy, dx = dy.reshape(-1), dx.reshape(-1)
    gam = D * 2.0 ** -24 * 1.0001
    for a in range(0, sel.size, chunk):
        q = sel[a:a + chunk]
        cy = cen[q, 1][:, None] + dy[None, :]
        cx = cen[q, 0][:, None] + dx[None, :]
        inb = (cy >= 0) & (cy < H) & (cx >= 0) & (cx < W)
        m = np.where(inb, cy * W + cx, 0)
        with np.errstate(invalid="ignore", over="ignore"):
            sc = np.einsum("qk,qck->qc", Dj[q], Di[m])
        sc = np.where(inb, sc, -np.inf)
        bad = ~np.isfinite(np.where(inb, sc, 0.0)).all(1)
        best = sc.max(1)
        arg = sc.argmax(1)
        g = qn[q] * gam
        hit = (m == flat_idx[q][:, None]) & inb
        found = hit.any(1)
        pos = hit.argmax(1)
        s_g = sc[np.arange(q.size), pos]
        tol = g * (dn[m[np.arange(q.size), pos]] + dn[m[np.arange(q.size), arg]]) + 1e-12
        ok[q] = found & (s_g >= best - tol)
        nonfin[q] = bad
    checked = np.asarray(mask).reshape(-1) & ~nonfin
    return ok.reshape(H, W), checked.reshape(H, W), nonfin.reshape(H, W)


def compare(gpu: dict, ora: dict, label: str = "", strict: bool = True, p_theta_max: float | None = None,
            pair=None, r: int | None = None, levels: int = 1) -> dict:
    """Compare one pair's outputs; returns the statistics (asserts if strict).

    p_theta_max: compare p* and theta only where the oracle's residual angle is
    at most this (for runs with the angle gate off, where matches beyond the
    image border are valid but their p* is not a zero-residual root).
    pair, r: the pair's descriptors and refine radius, for the per-query idx
    check of every good query (single-level refine only).
    """
    vg, vo = gpu["valid"], ora["valid"]
    both = vg & vo
    n = vg.size
    agree = float((vg == vo).mean())
    good = (ora["idx"] != -1) & (gpu["idx"] != -1)
    st = dict(label=label, queries=int(n), valid_oracle=int(vo.sum()), valid_gpu=int(vg.sum()),
              valid_both=int(both.sum()), valid_agreement=agree)
    cont = both if p_theta_max is None else both & (ora["theta"] <= p_theta_max)
    if "theta" in gpu:
        conv = good & (ora["theta"] <= CONVERGED_THETA) & (gpu["theta"] <= CONVERGED_THETA)
        st["p_compared_converged_not_both_valid"] = int((conv & ~cont).sum())
        cont = cont | conv
    if p_theta_max is not None:
        st["p_compared"] = int(cont.sum())
    if cont.any():
        dp = np.abs(gpu["p"] - ora["p"]).max(-1)[cont]
        st["max_dp_px"] = float(dp.max())
        if "theta" in gpu:
            st["max_dtheta"] = float(np.abs(gpu["theta"][cont] - ora["theta"][cont]).max())
    else:
        st.update(max_dp_px=0.0, max_dtheta=0.0)
    if "theta" in gpu and good.any():
        fin = good & np.isfinite(ora["theta"]) & np.isfinite(gpu["theta"])
        if fin.any():
            st["max_dtheta_all_good"] = float(np.abs(gpu["theta"][fin] - ora["theta"][fin]).max())
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
    if pair is not None and r is not None and levels == 1 and good.any():
        ok, checked, nonfin = idx_admissible(pair.Dii, pair.Dji, gpu["p"], gpu["idx"], r, good)
        st["idx_checked_all_good"] = int(checked.sum())
        st["idx_invalid"] = int((checked & ~ok).sum())
        if both.any():
            excl = both & ~comparable
            st["idx_excluded_checked"] = int((excl & checked).sum())
        st["idx_unchecked_nonfinite"] = int(nonfin.sum())
    # Queries the oracle rejects as bad input must be rejected the same way.
    bad = ora["idx"] == -1
    st["bad_input_mismatch"] = int(((gpu["idx"] != -1) | vg)[bad].sum())
    if strict:
        assert st["max_dp_px"] <= P_TOL, st
        assert st.get("max_dtheta", 0.0) <= THETA_TOL, st
        assert st.get("max_dtheta_all_good", 0.0) <= THETA_TOL, st
        assert st["idx_mismatch"] == 0, st
        assert st.get("idx_invalid", 0) == 0, st
        assert agree >= VALID_AGREE, st
        assert st["bad_input_mismatch"] == 0, st
    return st
