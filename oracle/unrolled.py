"""Vectorised fp64 torch-CPU restatement of the matcher's LM projection (test infrastructure).

An independent second statement of the geometric part of the matcher
(Sec. 3.2, Eq. 2 and Eq. 3; ray normalisation of Sec. 3.1) written with torch
tensor operations over all queries at once, so that torch autograd can
differentiate through the K unrolled Levenberg-Marquardt iterations.  The
tests use it two ways:

* its p* and theta must agree with the C oracle to fp64 rounding (the two
  share no code), and
* its autograd gradient of a loss through the unrolled solve must agree with
  the C oracle's implicit adjoint once the iterations have converged.

It follows the same readings as the C oracle: pixel centres at integers,
bilinear sampling of the normalised ray image with renormalisation, the
Jacobian from bilinear samples of central-difference gradient images, fixed K,
Levenberg damping x10 / /10 with acceptance on strictly lower cost, clamping
to the image domain with a coordinate held on its bound when its step points
outward.  Accept/reject decisions are taken on values and enter
autograd through ``torch.where``; floor() of the cell origin is piecewise
constant.  Inputs are assumed finite with non-zero points.
"""
from __future__ import annotations

import torch


def ray_image(X: torch.Tensor) -> torch.Tensor:
    """psi(X) = X / |X| per pixel (Sec. 3.1)."""
    return X / torch.linalg.norm(X, dim=-1, keepdim=True)


def gradient_images(R: torch.Tensor):
    """Central differences along x and y, one-sided at the border."""
    H, W, _ = R.shape
    xp = torch.clamp(torch.arange(W) + 1, max=W - 1)
    xm = torch.clamp(torch.arange(W) - 1, min=0)
    yp = torch.clamp(torch.arange(H) + 1, max=H - 1)
    ym = torch.clamp(torch.arange(H) - 1, min=0)
    Gx = (R[:, xp] - R[:, xm]) / (xp - xm).to(R.dtype)[None, :, None]
    Gy = (R[yp] - R[ym]) / (yp - ym).to(R.dtype)[:, None, None]
    return Gx, Gy


def _bilinear(img: torch.Tensor, x0, y0, a, b):
    """Bilinear sample of an (H, W, C) image at cell (x0, y0) with weights (a, b)."""
    f = lambda yy, xx: img[yy, xx]
    a = a[:, None]
    b = b[:, None]
    return ((1 - a) * (1 - b) * f(y0, x0) + a * (1 - b) * f(y0, x0 + 1)
            + (1 - a) * b * f(y0 + 1, x0) + a * b * f(y0 + 1, x0 + 1))


def _cell(p: torch.Tensor, H: int, W: int):
    x0 = torch.clamp(torch.floor(p[:, 0].detach()), 0, W - 2).long()
    y0 = torch.clamp(torch.floor(p[:, 1].detach()), 0, H - 2).long()
    return x0, y0, p[:, 0] - x0.to(p.dtype), p[:, 1] - y0.to(p.dtype)


def _sample(R, Gx, Gy, p, t):
    H, W, _ = R.shape
    x0, y0, a, b = _cell(p, H, W)
    r = _bilinear(R, x0, y0, a, b)
    gx = _bilinear(Gx, x0, y0, a, b)
    gy = _bilinear(Gy, x0, y0, a, b)
    n = torch.linalg.norm(r, dim=-1, keepdim=True)
    psi = r / n
    Jx = (gx - psi * (psi * gx).sum(-1, keepdim=True)) / n
    Jy = (gy - psi * (psi * gy).sum(-1, keepdim=True)) / n
    e = psi - t
    return (e * e).sum(-1), e, Jx, Jy


def lm_project(Xii: torch.Tensor, Xji: torch.Tensor, K: int = 10, lambda0: float = 1e-8,
               p_init: torch.Tensor | None = None):
    """Unrolled LM of Eq. 2 for every query; returns p* (N, 2), theta (N,), xhat (N, 3)."""
    H, W, _ = Xii.shape
    R = ray_image(Xii)
    Gx, Gy = gradient_images(R)
    x = Xji.reshape(-1, 3)
    t = x / torch.linalg.norm(x, dim=-1, keepdim=True)
    N = x.shape[0]
    if p_init is None:
        ys, xs = torch.meshgrid(torch.arange(H, dtype=Xii.dtype), torch.arange(W, dtype=Xii.dtype), indexing="ij")
        p = torch.stack([xs.reshape(-1), ys.reshape(-1)], -1)
    else:
        p = p_init.reshape(N, 2).to(Xii.dtype)
    lo = torch.zeros(2, dtype=Xii.dtype)
    hi = torch.tensor([W - 1.0, H - 1.0], dtype=Xii.dtype)
    p = torch.minimum(torch.maximum(p, lo), hi)
    c, e, Jx, Jy = _sample(R, Gx, Gy, p, t)
    lam = torch.full((N,), float(lambda0), dtype=Xii.dtype)
    for _ in range(K):
        a00 = (Jx * Jx).sum(-1) + lam
        a01 = (Jx * Jy).sum(-1)
        a11 = (Jy * Jy).sum(-1) + lam
        g0 = (Jx * e).sum(-1)
        g1 = (Jy * e).sum(-1)
        det = a00 * a11 - a01 * a01
        dx = -(a11 * g0 - a01 * g1) / det
        dy = -(a00 * g1 - a01 * g0) / det
        # Bounds: hold a coordinate on its bound whose step points outward; the
        # other then takes its 1-D damped step.
        hx = (((p[:, 0] <= 0) & (dx < 0)) | ((p[:, 0] >= W - 1) & (dx > 0))).detach()
        hy = (((p[:, 1] <= 0) & (dy < 0)) | ((p[:, 1] >= H - 1) & (dy > 0))).detach()
        zero = torch.zeros_like(dx)
        dx, dy = (torch.where(hx, zero, torch.where(hy, -g0 / a00, dx)),
                  torch.where(hy, zero, torch.where(hx, -g1 / a11, dy)))
        d = torch.stack([dx, dy], -1)
        q = torch.minimum(torch.maximum(p + d, lo), hi)
        cq, eq, Jxq, Jyq = _sample(R, Gx, Gy, q, t)
        acc = (cq < c).detach()
        p = torch.where(acc[:, None], q, p)
        c = torch.where(acc, cq, c)
        e = torch.where(acc[:, None], eq, e)
        Jx = torch.where(acc[:, None], Jxq, Jx)
        Jy = torch.where(acc[:, None], Jyq, Jy)
        lam = torch.where(acc, lam / 10.0, lam * 10.0)
    theta = 2.0 * torch.asin(torch.clamp(torch.sqrt(c) / 2.0, max=1.0))
    x0, y0, a, b = _cell(p, H, W)
    xhat = _bilinear(Xii, x0, y0, a, b)
    return p, theta, xhat
