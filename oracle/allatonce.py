"""The all-at-once system of Section 1: T u = f (eq. (1.2)) and its time-reversed
symmetric form Y T u = Y f (eqs. (1.3)-(1.4)).

Test infrastructure only (see ``oracle/__init__``).

Vectors are numpy arrays of shape [nt] + level_shape: the block u^(k) of eq. (1.2)
(k = 1..nt) is row k-1 of the array.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import Grid, L_matrix


def time_band_matrices(nt: int):
    """The n x n banded Toeplitz factors of T: T = B1 (x) L + B2 (x) (-2 I_m) with
    B1 = I + (shift)^2 and B2 = shift (alpha = 0 in eq. (1.6))."""
    Z = sp.diags([np.ones(nt - 1)], [-1], shape=(nt, nt), format="csr")
    B1 = (sp.identity(nt) + Z @ Z).tocsr()
    return B1, Z


def assemble_T(g: Grid) -> sp.csr_matrix:
    """Assemble the mn x mn block lower-triangular Toeplitz matrix T of eq. (1.2):
    block rows (L), (-2I, L), (L, -2I, L), ...  Sparse; small sizes only."""
    L = L_matrix(g)
    B1, Z = time_band_matrices(g.nt)
    return (sp.kron(B1, L) + sp.kron(Z, -2.0 * sp.identity(g.m))).tocsr()


def assemble_Y(g: Grid) -> sp.csr_matrix:
    """Y = Y_n (x) I_m with Y_n the n x n anti-identity (after eq. (1.4))."""
    Yn = sp.csr_matrix(np.fliplr(np.eye(g.nt)))
    return sp.kron(Yn, sp.identity(g.m)).tocsr()


def apply_T(g: Grid, u: np.ndarray, L=None) -> np.ndarray:
    """Matrix-free T u: (T u)^(k) = L u^(k) - 2 u^(k-1) + L u^(k-2), with the terms
    of non-existent levels (k-1 < 1, k-2 < 1) dropped, as in eq. (1.2)."""
    L = L_matrix(g) if L is None else L
    n = g.nt
    U = u.reshape(n, g.m)
    LU = (L @ U.T).T
    out = LU.copy()
    out[1:] -= 2.0 * U[:-1]
    out[2:] += LU[:-2]
    return out.reshape(g.shape)


def reverse_time(v: np.ndarray) -> np.ndarray:
    """Y v: reverse the order of the nt time levels (after eq. (1.4))."""
    return v[::-1].copy()


def apply_A(g: Grid, u: np.ndarray, L=None) -> np.ndarray:
    """A u = Y T u, the symmetric matrix of eq. (1.4)."""
    return reverse_time(apply_T(g, u, L))


def build_rhs(g: Grid, src: np.ndarray, psi0: np.ndarray, psi1: np.ndarray) -> np.ndarray:
    """Right-hand side f of eq. (1.2).

    ``src`` holds the source samples f^(0..nt-1) (shape [nt] + level_shape),
    ``psi0``/``psi1`` the initial displacement and velocity on the grid.  As printed:
        block 1: tau^2 f^(0)/2 + tau psi_1 + psi_0
        block 2: tau^2 f^(1) - L psi_0
        block k: tau^2 f^(k-1),  k = 3..nt.
    (A ghost-point derivation would give tau L psi_1 in block 1; the printed form
    is taken because it reproduces Table 2 of Section 3.)
    """
    tau2 = g.tau ** 2
    f = tau2 * np.asarray(src, dtype=np.float64).copy()
    f[0] = 0.5 * tau2 * src[0] + g.tau * psi1 + psi0
    L = L_matrix(g)
    f[1] = tau2 * src[1] - (L @ np.asarray(psi0).reshape(-1)).reshape(g.level_shape)
    return f


def solve_time_stepping(g: Grid, f: np.ndarray) -> np.ndarray:
    """Exact (to rounding) solution of T u = f by forward block substitution, i.e.
    the implicit leap-frog scheme marched level by level with a sparse LU of L:
        L u1 = f1;  L u2 = f2 + 2 u1;  L uk = fk + 2 u(k-1) - L u(k-2).
    An algorithm independent of any Krylov solver, used to pin MINRES results."""
    L = L_matrix(g).tocsc()
    lu = spla.splu(L)
    n = g.nt
    F = f.reshape(n, g.m)
    U = np.zeros_like(F)
    for k in range(n):
        rhs = F[k].copy()
        if k >= 1:
            rhs += 2.0 * U[k - 1]
        if k >= 2:
            rhs -= L @ U[k - 2]
        U[k] = lu.solve(rhs)
    return U.reshape(g.shape)
