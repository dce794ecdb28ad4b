"""Preconditioned MINRES for A x = b with A symmetric and an SPD preconditioner P
given through its inverse (the solver of Section 3, preconditioned system eq. (1.10)).

Test infrastructure only (see ``oracle/__init__``).

The method is the Lanczos process in the P^{-1} inner product followed by an
incrementally updated QR factorisation of the tridiagonal Lanczos matrix with Givens
rotations (Paige and Saunders' MINRES; the convergence lemma of Section 2.2 is the
estimate of Elman, Silvester and Wathen, Theorem 6.13).  Steps, in order, for
iteration j = 1, 2, ...:

  Lanczos:   q = A z_j;  delta_j = <q, z_j>;  q -= delta_j v_j + gamma_j v_{j-1};
             p = P^{-1} q;  gamma_{j+1} = sqrt(<q, p>);
             v_{j+1} = q / gamma_{j+1};  z_{j+1} = p / gamma_{j+1}
  QR:        apply rotation j-2 then j-1 to the new column (gamma_j, delta_j),
             form rotation j from (t2, gamma_{j+1})
  update:    w_j = (z_j - delta' w_{j-1} - eps w_{j-2}) / rho_j
             x_j = x_{j-1} + c_j eta w_j;   eta <- -s_j eta
  residual:  r_j = s_j^2 r_{j-1} - s_j c_j eta_{j-1} v_{j+1}   (true residual b - A x_j)

with v_1 = b / gamma_1, z_1 = P^{-1} b / gamma_1, gamma_1 = sqrt(<b, P^{-1} b>),
eta_0 = gamma_1, x_0 = 0.

Stopping rule (reading of Section 3: "relative residual norms", ||r_k||_2 <= tol):
stop at the first j with ||r_j||_2 <= tol * ||b||_2, the unpreconditioned 2-norm of
the residual of Y T u = Y f.  One iteration = one A apply and one P^{-1} apply;
the initial P^{-1} b is not counted.  This rule reproduces the iteration counts of
Table 1.  After the recurrence says "converged", the residual is recomputed
explicitly; if that fails the test the iteration continues with explicit checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class MinresResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float                       # explicit ||b - A x|| / ||b||
    relres_history: list = field(default_factory=list)   # recurrence ||r_j||/||b||, j = 0..iters
    eta_history: list = field(default_factory=list)      # |eta_j| (P^{-1}-norm of residual)
    breakdown: bool = False


def minres(apply_A, apply_Pinv, b: np.ndarray, tol: float = 1e-8, maxit: int = 1000,
           fixed_iters: int | None = None, stop: str = "true") -> MinresResult:
    """Preconditioned MINRES with zero initial guess.

    ``fixed_iters``: run exactly that many iterations (no stopping test), used to
    compare iterates x_k.  ``stop``: "true" (default; unpreconditioned 2-norm
    residual) or "precond" (|eta_j| <= tol * gamma_1, the P^{-1}-norm), the latter
    only to document that it does not reproduce Table 1.
    """
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    b = b.reshape(-1)
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return MinresResult(x.reshape(shape), 0, True, 0.0, [0.0], [0.0])

    r = b.copy()
    p = apply_Pinv(b.reshape(shape)).reshape(-1)
    gamma2 = float(b @ p)
    if not (gamma2 > 0.0 and math.isfinite(gamma2)):
        return MinresResult(x.reshape(shape), 0, False, 1.0, [1.0], [], breakdown=True)
    gamma = math.sqrt(gamma2)               # gamma_1
    v_prev = np.zeros_like(b)
    v = b / gamma
    z = p / gamma
    w_prev = np.zeros_like(b)               # w_{j-1}
    w_prev2 = np.zeros_like(b)              # w_{j-2}
    c_prev, c_prev2 = 1.0, 1.0              # c_{j-1}, c_{j-2}
    s_prev, s_prev2 = 0.0, 0.0              # s_{j-1}, s_{j-2}
    eta = gamma
    hist = [1.0]
    eta_hist = [abs(eta)]
    explicit_mode = False
    nmax = fixed_iters if fixed_iters is not None else maxit
    j = 0
    converged = False
    breakdown = False
    while j < nmax:
        j += 1
        # Lanczos step in the P^{-1} inner product
        q = apply_A(z.reshape(shape)).reshape(-1)
        delta = float(q @ z)
        q = q - delta * v - gamma * v_prev
        p = apply_Pinv(q.reshape(shape)).reshape(-1)
        gamma2_next = float(q @ p)
        if not math.isfinite(gamma2_next) or gamma2_next < 0.0:
            breakdown = True
            break
        gamma_next = math.sqrt(gamma2_next)
        # previous rotations applied to the new column (gamma_j, delta_j)
        eps = s_prev2 * gamma
        dbar = c_prev2 * gamma
        delta_p = c_prev * dbar + s_prev * delta
        t2 = -s_prev * dbar + c_prev * delta
        rho = math.hypot(t2, gamma_next)
        if rho == 0.0:
            breakdown = True
            break
        c = t2 / rho
        s = gamma_next / rho
        # solution update
        w = (z - delta_p * w_prev - eps * w_prev2) / rho
        x = x + (c * eta) * w
        # residual recurrence and next Lanczos vectors
        if gamma_next > 0.0:
            v_next = q / gamma_next
            z_next = p / gamma_next
        else:
            v_next = np.zeros_like(q)
            z_next = np.zeros_like(p)
        r = (s * s) * r - (s * c * eta) * v_next
        eta = -s * eta
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        eta_hist.append(abs(eta))
        # shift
        v_prev, v = v, v_next
        z = z_next
        w_prev2, w_prev = w_prev, w
        c_prev2, c_prev = c_prev, c
        s_prev2, s_prev = s_prev, s
        gamma = gamma_next
        if fixed_iters is not None:
            continue
        if stop == "precond":
            hit = abs(eta) <= tol * eta_hist[0]
        else:
            hit = rel <= tol
        if explicit_mode or hit:
            res = float(np.linalg.norm(b - apply_A(x.reshape(shape)).reshape(-1))) / bnorm
            ok = res <= tol if stop == "true" else hit
            if ok:
                converged = True
                break
            explicit_mode = True
        if gamma_next == 0.0:
            break
    relres = float(np.linalg.norm(b - apply_A(x.reshape(shape)).reshape(-1))) / bnorm
    if fixed_iters is not None:
        converged = relres <= tol
    return MinresResult(x.reshape(shape), j, converged, relres, hist, eta_hist, breakdown)


def krylov_minimiser(A: np.ndarray, Pinv: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
    """Brute force: the k-th preconditioned MINRES iterate (x_0 = 0) is the unique
    x in K_k(P^{-1}A, P^{-1}b) minimising ||b - A x||_{P^{-1}}.  Builds that Krylov
    basis explicitly (orthonormalised in the Euclidean inner product for stability)
    and solves the small least-squares problem through a Cholesky factor of P^{-1}.
    Dense, tiny sizes only."""
    b = b.reshape(-1)
    n = b.size
    M = Pinv @ A
    K = np.zeros((n, k))
    v = Pinv @ b
    for i in range(k):
        for jj in range(i):          # two passes of Gram-Schmidt
            v = v - (K[:, jj] @ v) * K[:, jj]
        for jj in range(i):
            v = v - (K[:, jj] @ v) * K[:, jj]
        K[:, i] = v / np.linalg.norm(v)
        v = M @ K[:, i]
    C = np.linalg.cholesky(0.5 * (Pinv + Pinv.T))      # Pinv = C C^T
    # ||b - A K y||_{P^{-1}}^2 = ||C^T (b - A K y)||_2^2
    G = C.T @ (A @ K)
    rhs = C.T @ b
    y, *_ = np.linalg.lstsq(G, rhs, rcond=None)
    return K @ y


def exact_minres_count(apply_A, b: np.ndarray, tol: float, kmax: int):
    """The exact-arithmetic MINRES (x_0 = 0, no preconditioner) iteration count: the
    smallest k with min over x in K_k(A, b) of ||b - A x||_2 <= tol ||b||_2.  Builds an
    orthonormal basis of K_k by Arnoldi with two Gram-Schmidt passes (no loss of
    orthogonality, unlike the three-term recurrence); the least-squares residual of the
    Hessenberg problem comes from its QR factorisation by Givens rotations, updated one
    column at a time.  Returns None if kmax steps do not suffice.  Finite-precision
    MINRES needs about this many steps or more; the delay beyond it comes from the loss
    of orthogonality of the short recurrence."""
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    n = b.size
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return 0
    Q = np.zeros((n, kmax + 1))
    Q[:, 0] = b / beta
    cs, sn = [], []
    g = beta                      # last entry of Q_k^T beta e_1 (the residual norm)
    for k in range(kmax):
        v = np.asarray(apply_A(Q[:, k]), dtype=np.float64).reshape(-1).copy()
        h = np.zeros(k + 2)
        for _ in range(2):
            hh = Q[:, :k + 1].T @ v
            v -= Q[:, :k + 1] @ hh
            h[:k + 1] += hh
        h[k + 1] = np.linalg.norm(v)
        for i in range(k):        # earlier rotations on the new column
            t = cs[i] * h[i] + sn[i] * h[i + 1]
            h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1]
            h[i] = t
        r = math.hypot(h[k], h[k + 1])
        c, s = (h[k] / r, h[k + 1] / r) if r > 0.0 else (1.0, 0.0)
        cs.append(c)
        sn.append(s)
        g = -s * g
        if abs(g) <= tol * beta:
            return k + 1
        if h[k + 1] == 0.0:
            return None
        Q[:, k + 1] = v / h[k + 1]
    return None
