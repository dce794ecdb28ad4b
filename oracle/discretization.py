"""Spatial grid and operators of the implicit leap-frog scheme (Section 1).

Test infrastructure only (see ``oracle/__init__``).

Grid: Omega = (0,1)^d, d in {1, 2}; interior points x_i = i*h, i = 1..nx, with
h = 1/(nx+1) (and hy = 1/(ny+1) in 2D).  Unknowns of one time level are stored in
lexicographic order with x fastest, i.e. a 2D level is an array [ny][nx].
Homogeneous Dirichlet data: ghost values outside the grid are zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.fft as sfft


class Grid:
    """Space-time grid.  ``ny == 0`` selects the 1D problem.

    tau = T/nt is the time step of the scheme (Section 1); the unknown levels are
    t_k = k*tau, k = 1..nt, and level 0 carries the initial data psi_0.
    """

    def __init__(self, nx: int, ny: int, nt: int, T: float = 1.0):
        if nx < 1 or ny < 0 or nt < 2 or not T > 0:
            raise ValueError("bad grid")
        self.nx, self.ny, self.nt, self.T = int(nx), int(ny), int(nt), float(T)
        self.hx = 1.0 / (nx + 1)
        self.hy = 1.0 / (ny + 1) if ny else None
        self.tau = self.T / nt

    @property
    def dim(self) -> int:
        return 2 if self.ny else 1

    @property
    def level_shape(self) -> tuple:
        return (self.ny, self.nx) if self.ny else (self.nx,)

    @property
    def shape(self) -> tuple:
        """Shape of one all-at-once vector: [nt] + level_shape."""
        return (self.nt,) + self.level_shape

    @property
    def m(self) -> int:
        """Spatial unknowns per level."""
        return self.nx * (self.ny if self.ny else 1)

    @property
    def N(self) -> int:
        return self.m * self.nt

    def points(self):
        """Interior coordinates: (x,) in 1D, (X, Y) meshgrids of shape [ny][nx] in 2D."""
        x = self.hx * np.arange(1, self.nx + 1)
        if not self.ny:
            return (x,)
        y = self.hy * np.arange(1, self.ny + 1)
        X, Y = np.meshgrid(x, y, indexing="xy")
        return (X, Y)

    def times(self):
        """t_k = k*tau for k = 0..nt (level 0 is the initial time)."""
        return self.tau * np.arange(self.nt + 1)


def second_difference(n: int, h: float) -> sp.csr_matrix:
    """Dirichlet 3-point second difference tridiag(1, -2, 1)/h^2 of size n."""
    e = np.ones(n)
    return sp.diags([e[:-1], -2.0 * e, e[:-1]], [-1, 0, 1], format="csr") / (h * h)


def laplacian(g: Grid) -> sp.csr_matrix:
    """Delta_h: the 3-point (1D) or 5-point (2D) Laplacian with homogeneous
    Dirichlet conditions, in lexicographic (x fastest) order (Section 1)."""
    Dx = second_difference(g.nx, g.hx)
    if not g.ny:
        return Dx
    Dy = second_difference(g.ny, g.hy)
    return (sp.kron(sp.identity(g.ny), Dx) + sp.kron(Dy, sp.identity(g.nx))).tocsr()


def L_matrix(g: Grid, abar: float = 1.0) -> sp.csr_matrix:
    """L = I_m - (tau^2/2) Delta_h, the diagonal block of T in eq. (1.2); with abar,
    the mean-coefficient block L_abar = I_m - (abar tau^2/2) Delta_h of eq. (3.3)."""
    return (sp.identity(g.m) - 0.5 * abar * g.tau ** 2 * laplacian(g)).tocsr()


def neg_laplacian_eigenvalues(g: Grid) -> np.ndarray:
    """Eigenvalues kappa of -Delta_h in the sine basis, shaped like one level.

    1D: kappa_j = (4/h^2) sin^2(j*pi*h/2), j = 1..nx.  2D: the sum over the two
    axes, indexed [jy][jx].  These are the entries of the diagonal Lambda in
    L = U Lambda U^T of Section 2.3 once mapped through L = I + tau^2/2 (-Delta_h).
    """
    jx = np.arange(1, g.nx + 1)
    kx = (4.0 / g.hx ** 2) * np.sin(jx * np.pi * g.hx / 2.0) ** 2
    if not g.ny:
        return kx
    jy = np.arange(1, g.ny + 1)
    ky = (4.0 / g.hy ** 2) * np.sin(jy * np.pi * g.hy / 2.0) ** 2
    return ky[:, None] + kx[None, :]


def L_eigenvalues(g: Grid, abar: float = 1.0) -> np.ndarray:
    """lambda_j(L) = 1 + (abar tau^2/2) kappa_j, shaped like one level (abar = 1: eq.
    (1.2); otherwise the mean-coefficient block of eq. (3.3))."""
    return 1.0 + 0.5 * abar * g.tau ** 2 * neg_laplacian_eigenvalues(g)


def dst_space(v: np.ndarray, g: Grid) -> np.ndarray:
    """Apply the orthonormal (multi-dimensional) DST-I, the matrix U = S of
    Section 2.3, to every time level of ``v`` (shape [..., nt] + level_shape).

    S is real, symmetric and orthogonal, so it is its own inverse.  This calls the
    scipy.fft DST-I routine, a library primitive (on every host core: the threads
    split the batch of transforms, so the result does not depend on their number).
    """
    axes = (-2, -1) if g.ny else (-1,)
    return sfft.dstn(v, type=1, axes=axes, norm="ortho", workers=-1)


def dst_matrix(n: int) -> np.ndarray:
    """Dense orthonormal DST-I matrix sqrt(2/(n+1)) sin(pi j k/(n+1)), j,k = 1..n."""
    j = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(j, j) / (n + 1))
