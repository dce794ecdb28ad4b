"""Restarted GMRES with right preconditioning, for the non-symmetric all-at-once system
T u = f with the block alpha-circulant preconditioner C_alpha (eqs. (1.2), (1.5)-(1.7);
the preconditioner of the prior work the paper starts from, which needs a
non-symmetric Krylov solver because C_alpha is not symmetric).

Test infrastructure only (see ``oracle/__init__``).

GMRES (Saad and Schultz) with right preconditioning M = C_alpha^{-1}: the k-th iterate
is x_k = x_0 + M V_k y_k, where V_k is an orthonormal basis of the Krylov space
K_k(A M, r_0) built by the Arnoldi process (modified Gram-Schmidt), and y_k minimises
|| beta e_1 - H_k y || for the (k+1) x k Hessenberg matrix H_k, solved through Givens
rotations.  With right preconditioning the minimised quantity is the true residual
||b - A x_k||_2, so the stopping rule is the one of the MINRES solver (Section 3):
stop at the first k with ||b - A x_k||_2 <= tol ||b||_2 (the rotated residual), then
confirm it explicitly; if the confirmation fails, restart.  A cycle ends after
`restart` steps; the next cycle starts from the explicit residual.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float                                   # explicit ||b - A x|| / ||b||
    relres_history: list = field(default_factory=list)   # rotated residual / ||b|| per step


def gmres(apply_A, apply_Minv, b: np.ndarray, tol: float = 1e-8, maxit: int = 1000, restart: int = 30,
          fixed_iters: int | None = None) -> GmresResult:
    """Right-preconditioned restarted GMRES with zero initial guess.  ``fixed_iters``
    runs exactly that many steps (restarts included) with no stopping test."""
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    bv = b.reshape(-1)
    A = lambda v: np.asarray(apply_A(v.reshape(shape)), dtype=np.float64).reshape(-1)
    M = lambda v: np.asarray(apply_Minv(v.reshape(shape)), dtype=np.float64).reshape(-1)
    bnorm = float(np.linalg.norm(bv))
    x = np.zeros_like(bv)
    hist = [1.0]
    if bnorm == 0.0:
        return GmresResult(x.reshape(shape), 0, True, 0.0, hist)
    nmax = fixed_iters if fixed_iters is not None else maxit
    k = 0
    converged = False
    while k < nmax:
        r = bv - A(x)
        beta = float(np.linalg.norm(r))
        if fixed_iters is None and beta <= tol * bnorm:
            converged = True
            break
        m = min(restart, nmax - k)
        V = np.zeros((bv.size, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        hit = False
        for j in range(m):
            w = A(M(V[:, j]))
            for l in range(j + 1):                 # modified Gram-Schmidt
                H[l, j] = float(w @ V[:, l])
                w = w - H[l, j] * V[:, l]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for l in range(j):                     # earlier rotations on the new column
                t = cs[l] * H[l, j] + sn[l] * H[l + 1, j]
                H[l + 1, j] = -sn[l] * H[l, j] + cs[l] * H[l + 1, j]
                H[l, j] = t
            rho = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / rho, H[j + 1, j] / rho) if rho > 0.0 else (1.0, 0.0)
            H[j, j] = rho
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            k += 1
            j_done = j + 1
            hist.append(abs(gvec[j + 1]) / bnorm)
            if fixed_iters is None and abs(gvec[j + 1]) <= tol * bnorm:
                hit = True
                break
            if H[j + 1, j] == 0.0 and rho == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), gvec[:j_done])
        x = x + M(V[:, :j_done] @ y)
        if hit:
            res = float(np.linalg.norm(bv - A(x))) / bnorm
            if res <= tol:
                converged = True
                break
    relres = float(np.linalg.norm(bv - A(x))) / bnorm
    if fixed_iters is not None:
        converged = relres <= tol
    return GmresResult(x.reshape(shape), k, converged, relres, hist)


def krylov_minimiser_right(A: np.ndarray, Minv: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
    """Brute force: the k-th right-preconditioned GMRES iterate (x_0 = 0) is
    M y with y in K_k(A M, b) minimising ||b - A M y||_2.  Builds that Krylov basis
    explicitly (two Gram-Schmidt passes) and solves the small least-squares problem.
    Dense, tiny sizes only."""
    b = b.reshape(-1)
    AM = A @ Minv
    K = np.zeros((b.size, k))
    v = b.copy()
    for i in range(k):
        for _ in range(2):
            for jj in range(i):
                v = v - (K[:, jj] @ v) * K[:, jj]
        K[:, i] = v / np.linalg.norm(v)
        v = AM @ K[:, i]
    c, *_ = np.linalg.lstsq(AM @ K, b, rcond=None)
    return Minv @ (K @ c)
