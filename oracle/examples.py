"""Example 1 of Section 3 and the error measure E_{tau,h}.

Test infrastructure only (see ``oracle/__init__``).

Example 1 (d = 2, Omega = (0,1)^2, T = 1): exact solution
u(x, t) = exp(-t) x1 (x1 - 1) x2 (x2 - 1); psi_0 = -psi_1 = x1 (x1-1) x2 (x2-1);
f = exp(-t) (x1(x1-1) x2(x2-1) - 2 (x1(x1-1) + x2(x2-1))).
"""
from __future__ import annotations

import numpy as np

from .discretization import Grid


def example1_data(g: Grid):
    """Source samples f^(0..nt-1), psi_0, psi_1 and the exact solution at levels
    1..nt for Example 1 (2D only)."""
    if g.dim != 2:
        raise ValueError("Example 1 is two-dimensional")
    X, Y = g.points()
    phi = X * (X - 1.0) * Y * (Y - 1.0)
    lap = 2.0 * (X * (X - 1.0) + Y * (Y - 1.0))
    t = g.times()
    src = np.exp(-t[:-1])[:, None, None] * (phi - lap)[None]
    psi0 = phi.copy()
    psi1 = -phi.copy()
    exact = np.exp(-t[1:])[:, None, None] * phi[None]
    return src, psi0, psi1, exact


def error_E(g: Grid, u: np.ndarray, exact: np.ndarray) -> float:
    """E_{tau,h} = max_k h^{d/2} ||u^(k) - u(G_h, k tau)||_2 (Section 3)."""
    d = g.dim
    diff = (u - exact).reshape(g.nt, -1)
    return float(np.max(g.hx ** (d / 2.0) * np.linalg.norm(diff, axis=1)))
