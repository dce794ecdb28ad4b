"""Variable-coefficient wave equation u_tt = div(a grad u) + f (Section 3, eq. (3.1)):
the all-at-once matrix with blocks L_a (eq. (3.2)) and the mean-coefficient
preconditioner built from L_abar, abar = mean of a over the grid points (eq. (3.3)).

Test infrastructure only (see ``oracle/__init__``).

Readings taken (each recorded with the tests that pin them):
* Delta_{a,h} is the conservative 5-point (3-point in 1D) central difference of
  div(a grad u) with a evaluated at the cell midpoints:
  (Delta_{a,h} u)_i = [a_{i+1/2}(u_{i+1} - u_i) - a_{i-1/2}(u_i - u_{i-1})]/h^2 per axis,
  which keeps L_a symmetric (MINRES needs Y T symmetric);
* the second right-hand-side row uses L_a psi_0 (the block of the scheme), where eq.
  (3.2) prints the constant-coefficient symbol.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .discretization import Grid


def coefficient_samples(g: Grid, afun):
    """a at the interior points ([ny][nx] or [nx]), at the x half points
    x_{i+1/2}, i = 0..nx ([ny1][nx+1]) and, in 2D, at the y half points ([ny+1][nx])."""
    x = g.hx * np.arange(1, g.nx + 1)
    xh = g.hx * (np.arange(0, g.nx + 1) + 0.5)
    if not g.ny:
        return afun(x), afun(xh)[None, :], None
    y = g.hy * np.arange(1, g.ny + 1)
    yh = g.hy * (np.arange(0, g.ny + 1) + 0.5)
    X, Y = np.meshgrid(x, y, indexing="xy")
    Xh, Yx = np.meshgrid(xh, y, indexing="xy")
    Xy, Yh = np.meshgrid(x, yh, indexing="xy")
    return afun(X, Y), afun(Xh, Yx), afun(Xy, Yh)


def laplacian_var(g: Grid, a_xh: np.ndarray, a_yh) -> sp.csr_matrix:
    """Conservative central difference of div(a grad .) with zero Dirichlet data."""
    nx, ny1 = g.nx, (g.ny if g.ny else 1)
    rows, cols, vals = [], [], []

    def idx(i, j):
        return j * nx + i

    for j in range(ny1):
        for i in range(nx):
            c = idx(i, j)
            aw, ae = a_xh[j, i], a_xh[j, i + 1]
            diag = -(aw + ae) / g.hx ** 2
            if i > 0:
                rows.append(c); cols.append(idx(i - 1, j)); vals.append(aw / g.hx ** 2)
            if i < nx - 1:
                rows.append(c); cols.append(idx(i + 1, j)); vals.append(ae / g.hx ** 2)
            if g.ny:
                as_, an = a_yh[j, i], a_yh[j + 1, i]
                diag -= (as_ + an) / g.hy ** 2
                if j > 0:
                    rows.append(c); cols.append(idx(i, j - 1)); vals.append(as_ / g.hy ** 2)
                if j < ny1 - 1:
                    rows.append(c); cols.append(idx(i, j + 1)); vals.append(an / g.hy ** 2)
            rows.append(c); cols.append(c); vals.append(diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.m, g.m))


def L_var(g: Grid, a_xh, a_yh) -> sp.csr_matrix:
    """L_a = I - (tau^2/2) Delta_{a,h} (eq. (3.2))."""
    return (sp.identity(g.m) - 0.5 * g.tau ** 2 * laplacian_var(g, a_xh, a_yh)).tocsr()


def apply_T_var(g: Grid, u: np.ndarray, La) -> np.ndarray:
    """(T_a u)^(k) = L_a u^(k) - 2 u^(k-1) + L_a u^(k-2) (eq. (3.2))."""
    U = u.reshape(g.nt, g.m)
    LU = (La @ U.T).T
    out = LU.copy()
    out[1:] -= 2.0 * U[:-1]
    out[2:] += LU[:-2]
    return out.reshape(g.shape)


def build_rhs_var(g: Grid, src, psi0, psi1, La) -> np.ndarray:
    """Right-hand side of eq. (3.2) (second row with L_a psi_0)."""
    tau2 = g.tau ** 2
    f = tau2 * np.asarray(src, dtype=np.float64).copy()
    f[0] = 0.5 * tau2 * src[0] + g.tau * psi1 + psi0
    f[1] = tau2 * src[1] - (La @ np.asarray(psi0).reshape(-1)).reshape(g.level_shape)
    return f


def example2_coefficient(x, y):
    """a(x) = (30 + sin^2 x1)(30 + sin^2 x2) of Example 2."""
    return (30.0 + np.sin(x) ** 2) * (30.0 + np.sin(y) ** 2)


def example2_data(g: Grid):
    """Source samples f^(0..nt-1), psi_0 = psi_1 = x1(1-x1) x2(1-x2) and the exact
    solution u = exp(t) x1(1-x1) x2(1-x2) of Example 2 (Section 3)."""
    X, Y = g.points()
    phi = X * (1 - X) * Y * (1 - Y)
    a = example2_coefficient(X, Y)
    fs = (phi - np.sin(2 * X) * (30 + np.sin(Y) ** 2) * (1 - 2 * X) * Y * (1 - Y)
          - np.sin(2 * Y) * (30 + np.sin(X) ** 2) * (1 - 2 * Y) * X * (1 - X)
          + 2 * a * (X * (1 - X) + Y * (1 - Y)))
    t = g.times()
    src = np.exp(t[:-1])[:, None, None] * fs[None]
    exact = np.exp(t[1:])[:, None, None] * phi[None]
    return src, phi.copy(), phi.copy(), exact
