"""Independent patch-alignment solvers used to pin the inverse search.

TEST INFRASTRUCTURE ONLY (see ``dis_oracle``).  These solve the same patch
problem, the mean-normalised form of Eq. (1), by other routes:

* ``forward_additive_lk``: the forward-additive Lucas-Kanade iteration of
  Suppl. A (before the roles of image and template are swapped), which
  re-evaluates the warped-image gradient and the Hessian every iteration;
* ``brute_force``: exhaustive search of the objective over a displacement
  grid, refined in two passes.

Neither shares code with the inverse-compositional search they check; each
carries its own bilinear interpolation.
"""
from __future__ import annotations

import torch

F64 = torch.float64


def _interp_with_gradient(img: torch.Tensor, x: torch.Tensor, y: torch.Tensor):
    """Bilinear value and its exact partial derivatives, edge-clamped taps."""
    h, w = img.shape
    fx = torch.floor(x)
    fy = torch.floor(y)
    ax = x - fx
    ay = y - fy
    ix = fx.long()
    iy = fy.long()
    c0 = ix.clamp(0, w - 1)
    c1 = (ix + 1).clamp(0, w - 1)
    r0 = iy.clamp(0, h - 1)
    r1 = (iy + 1).clamp(0, h - 1)
    p00, p01 = img[r0, c0], img[r0, c1]
    p10, p11 = img[r1, c0], img[r1, c1]
    val = (1 - ay) * ((1 - ax) * p00 + ax * p01) + ay * ((1 - ax) * p10 + ax * p11)
    ddx = (1 - ay) * (p01 - p00) + ay * (p11 - p10)
    ddy = (1 - ax) * (p10 - p00) + ax * (p11 - p01)
    return val, ddx, ddy


def _patch_coords(x0: int, y0: int, ps: int):
    yy, xx = torch.meshgrid(torch.arange(ps, dtype=F64), torch.arange(ps, dtype=F64), indexing="ij")
    return (xx + x0).reshape(-1), (yy + y0).reshape(-1)


def objective(J0, J1, x0: int, y0: int, ps: int, u: torch.Tensor) -> torch.Tensor:
    """Mean-normalised SSD between the template at (x0, y0) and I1 at x + u,
    for a batch of displacements u [K, 2]."""
    X, Y = _patch_coords(x0, y0, ps)
    T = J0[Y.long(), X.long()]
    Tn = T - T.mean()
    Q, _, _ = _interp_with_gradient(J1, X[None, :] + u[:, 0:1], Y[None, :] + u[:, 1:2])
    Qn = Q - Q.mean(dim=1, keepdim=True)
    return ((Qn - Tn[None, :]) ** 2).sum(1)


def forward_additive_lk(J0, J1, x0: int, y0: int, ps: int, u0, iters: int = 100) -> torch.Tensor:
    """Gauss-Newton on the mean-normalised objective with the Jacobian of the
    warped image at the current u (forward-additive Lucas-Kanade)."""
    X, Y = _patch_coords(x0, y0, ps)
    T = J0[Y.long(), X.long()]
    Tn = T - T.mean()
    u = torch.as_tensor(u0, dtype=F64).clone()
    for _ in range(iters):
        Q, qx, qy = _interp_with_gradient(J1, X + u[0], Y + u[1])
        r = (Q - Q.mean()) - Tn
        sx = qx - qx.mean()
        sy = qy - qy.mean()
        H = torch.stack([torch.stack([(sx * sx).sum(), (sx * sy).sum()]),
                         torch.stack([(sx * sy).sum(), (sy * sy).sum()])])
        g = torch.stack([(sx * r).sum(), (sy * r).sum()])
        u = u - torch.linalg.solve(H, g)
    return u


def brute_force(J0, J1, x0: int, y0: int, ps: int, centre, radius: float = 1.5,
                step: float = 0.005) -> torch.Tensor:
    """Minimiser of ``objective`` on a grid: a 0.05 px pass over the square of
    half-width ``radius`` around ``centre``, then a ``step`` pass within
    +-0.1 px of the best point."""
    c = torch.as_tensor(centre, dtype=F64)

    def best_on(cx, cy, r, h):
        n = int(round(r / h))
        off = torch.arange(-n, n + 1, dtype=F64) * h
        gy, gx = torch.meshgrid(off + cy, off + cx, indexing="ij")
        cand = torch.stack([gx.reshape(-1), gy.reshape(-1)], 1)
        vals = torch.cat([objective(J0, J1, x0, y0, ps, cand[i:i + 8192])
                          for i in range(0, cand.shape[0], 8192)])
        return cand[int(torch.argmin(vals))]

    b = best_on(float(c[0]), float(c[1]), radius, 0.05)
    return best_on(float(b[0]), float(b[1]), 0.1, step)
