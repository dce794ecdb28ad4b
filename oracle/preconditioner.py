"""The block alpha-circulant matrix C_alpha and the ABAC preconditioner
P_alpha = (C_alpha^{1/2})^T C_alpha^{1/2} (Section 1, eqs. (1.5)-(1.9); Section 2.3).

Test infrastructure only (see ``oracle/__init__``).

Two tiers:

* dense (tiny sizes): C_alpha assembled from eq. (1.6), its principal square root by
  the library routine ``scipy.linalg.sqrtm`` (the definition of eq. (1.8)), P_alpha
  formed and inverted densely;
* matrix-free: the fast apply of Section 2.3, P^{-1} y = C^{-1/2} (C^{-1/2})^T y, as
  three steps (transform, diagonal, inverse transform) done twice, with complex FFTs
  in time and DST-I in space.  The transposed factor is applied as the transpose of
  the factorisation itself, not through any symmetry identity.  The FFT routines run
  on every host core (scipy.fft ``workers``); the threads split the batch of
  transforms, so the values do not depend on the core count.  Inputs are made complex
  before the time FFTs, so the complex transform runs even where the data are real.

Readings of the paper taken here (each pinned by a test):

* The alpha-circulant factors are diagonalised with numpy's DFT (exponent
  -2 pi i k t / n).  With D = diag(a^t), a = alpha^{1/n}, t = 0..n-1, the down-shift
  with alpha in its corner is Z_alpha = D^{-1} F^{-1} diag(a w_k) F D, w_k =
  exp(-2 pi i k / n).  The two printed forms (F Lambda F^* and F^* Lambda F) differ
  only in which eigenvalue is attached to which column; the spectrum is the same.
* The per-frequency block is Lambda_{alpha,1} (x) Lambda + Lambda_{alpha,2} (x) I_m,
  with the factor -2 counted once (it is already inside lambda_{2,k}), as in eq.
  (1.7) and Appendix A.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp

from .discretization import Grid, L_matrix, L_eigenvalues, dst_space
from .allatonce import assemble_T


def alpha_circulant_factors(nt: int, alpha: float):
    """B1^(alpha) and B2^(alpha) of eq. (1.6) (sparse, n x n)."""
    rows = list(range(1, nt)) + [0]
    cols = list(range(0, nt - 1)) + [nt - 1]
    vals = [1.0] * (nt - 1) + [alpha]
    Za = sp.csr_matrix((vals, (rows, cols)), shape=(nt, nt))
    B1 = sp.identity(nt) + Za @ Za
    return B1.tocsr(), Za


def assemble_C(g: Grid, alpha: float, abar: float = 1.0) -> sp.csr_matrix:
    """C_alpha = B1 (x) L + B2 (x) (-2 I_m), eqs. (1.5)-(1.6) (sparse); with abar the
    blocks are L_abar (eq. (3.3))."""
    L = L_matrix(g, abar)
    B1, B2 = alpha_circulant_factors(g.nt, alpha)
    return (sp.kron(B1, L) + sp.kron(B2, -2.0 * sp.identity(g.m))).tocsr()


def assemble_R(g: Grid, alpha: float) -> sp.csr_matrix:
    """R_alpha = C_alpha - T (Section 2.2)."""
    return (assemble_C(g, alpha) - assemble_T(g)).tocsr()


def time_eigenvalues(nt: int, alpha: float):
    """lambda_{1,k} = 1 + a^2 w_k^2 and lambda_{2,k} = -2 a w_k for k = 0..n-1, with
    a = alpha^{1/n} and w_k the eigenvalue of the cyclic down-shift for the k-th
    numpy DFT bin (eq. (1.7) and Section 2.3)."""
    a = alpha ** (1.0 / nt)
    w = np.exp(-2j * np.pi * np.arange(nt) / nt)
    return 1.0 + a * a * w * w, -2.0 * a * w


def mu_table(g: Grid, alpha: float, abar: float = 1.0) -> np.ndarray:
    """Eigenvalues mu_{k,j} = lambda_j(L) lambda_{1,k} + lambda_{2,k} of C_alpha
    (eq. (1.7); Appendix A), shaped [nt] + level_shape."""
    l1, l2 = time_eigenvalues(g.nt, alpha)
    lam = L_eigenvalues(g, abar)
    expand = (slice(None),) + (None,) * lam.ndim
    return lam[None, ...] * l1[expand] + l2[expand]


def principal_inv_sqrt(mu: np.ndarray) -> np.ndarray:
    """1/s(mu) with s the principal branch of the complex square root (eq. (1.8)).
    The spectrum avoids (-inf, 0] (Lemma on C_alpha in Section 2.1, Appendix A),
    which is asserted."""
    mu = np.asarray(mu, dtype=np.complex128)
    bad = (mu.real <= 0) & (mu.imag == 0)
    if np.any(bad):
        raise ValueError("C_alpha has an eigenvalue on (-inf, 0]")
    return 1.0 / np.sqrt(mu)


def time_scaling(nt: int, alpha: float) -> np.ndarray:
    """Diagonal of D_alpha = diag(alpha^{(i-1)/n}), i = 1..n (eq. (1.7))."""
    return alpha ** (np.arange(nt) / nt)


# --------------------------------------------------------------------------
# dense tier
# --------------------------------------------------------------------------

def dense_sqrt_C(g: Grid, alpha: float, abar: float = 1.0) -> np.ndarray:
    """C_alpha^{1/2} by scipy.linalg.sqrtm (Schur method, principal branch).
    Lemma on C_alpha in Section 2.1: the result is real; the imaginary part is
    checked small and dropped."""
    C = assemble_C(g, alpha, abar).toarray()
    S = sla.sqrtm(C)
    S = np.asarray(S)
    if np.iscomplexobj(S):
        if np.max(np.abs(S.imag)) > 1e-10 * max(1.0, np.max(np.abs(S.real))):
            raise AssertionError("principal square root of C_alpha is not real")
        S = S.real
    return S


def dense_P(g: Grid, alpha: float, abar: float = 1.0) -> np.ndarray:
    """P_alpha = (C_alpha^{1/2})^T C_alpha^{1/2} (eq. (1.9)), dense."""
    S = dense_sqrt_C(g, alpha, abar)
    return S.T @ S


def dense_apply_Pinv(g: Grid, alpha: float, y: np.ndarray, P=None) -> np.ndarray:
    """z = P_alpha^{-1} y by a dense symmetric positive definite solve."""
    P = dense_P(g, alpha) if P is None else P
    z = sla.solve(P, y.reshape(-1), assume_a="pos")
    return z.reshape(g.shape)


# --------------------------------------------------------------------------
# matrix-free tier: Section 2.3, three steps done twice
# --------------------------------------------------------------------------

def _time_axis_scale(v: np.ndarray, s: np.ndarray) -> np.ndarray:
    return v * s.reshape((-1,) + (1,) * (v.ndim - 1))


def apply_C_inv_sqrt_T(g: Grid, alpha: float, y: np.ndarray, abar: float = 1.0) -> np.ndarray:
    """(C_alpha^{-1/2})^T y.

    With C_alpha = (D^{-1} F^{-1} (x) S) diag(mu) (F D (x) S) (S = DST-I, F = DFT),
    the transposed inverse square root is (D F (x) S) diag(mu^{-1/2}) (F^{-1} D^{-1} (x) S):
      Step 1: DST in space, D^{-1} in time, inverse DFT in time;
      Step 2: multiply by mu^{-1/2};
      Step 3: DFT in time, D in time, DST in space.
    Returns a complex array whose imaginary part is rounding noise."""
    d = time_scaling(g.nt, alpha)
    M = principal_inv_sqrt(mu_table(g, alpha, abar))
    v = dst_space(np.asarray(y, dtype=np.float64), g)
    v = _time_axis_scale(v, 1.0 / d).astype(np.complex128)
    v = sfft.ifft(v, axis=0, workers=-1)
    v = M * v
    v = sfft.fft(v, axis=0, workers=-1)
    v = _time_axis_scale(v, d)
    return dst_space(v.real, g) + 1j * dst_space(v.imag, g)


def apply_C_inv_sqrt(g: Grid, alpha: float, y: np.ndarray, abar: float = 1.0) -> np.ndarray:
    """C_alpha^{-1/2} y = (D^{-1} F^{-1} (x) S) diag(mu^{-1/2}) (F D (x) S) y:
      Step 1: DST in space, D in time, DFT in time;
      Step 2: multiply by mu^{-1/2};
      Step 3: inverse DFT in time, D^{-1} in time, DST in space.
    Accepts and returns complex arrays."""
    d = time_scaling(g.nt, alpha)
    M = principal_inv_sqrt(mu_table(g, alpha, abar))
    y = np.asarray(y)
    v = dst_space(y.real, g) + 1j * dst_space(y.imag, g)
    v = _time_axis_scale(v, d)
    v = sfft.fft(v, axis=0, workers=-1)
    v = M * v
    v = sfft.ifft(v, axis=0, workers=-1)
    v = _time_axis_scale(v, 1.0 / d)
    return dst_space(v.real, g) + 1j * dst_space(v.imag, g)


def apply_Pinv(g: Grid, alpha: float, y: np.ndarray, check_imag: bool = True, abar: float = 1.0) -> np.ndarray:
    """z = P_alpha^{-1} y = C_alpha^{-1/2} (C_alpha^{-1/2})^T y (Section 2.3).

    The result is real (Lemma on C_alpha in Section 2.1); with ``check_imag`` the
    imaginary part is asserted to be rounding noise relative to the real part."""
    w = apply_C_inv_sqrt_T(g, alpha, y, abar)
    z = apply_C_inv_sqrt(g, alpha, w, abar)
    if check_imag:
        scale = max(np.max(np.abs(z.real)), 1e-300)
        imag = np.max(np.abs(z.imag))
        if imag > 1e-9 * scale:
            raise AssertionError(f"P^-1 y has a large imaginary part {imag:.3e} (scale {scale:.3e})")
    return z.real.copy()


def apply_C_inv(g: Grid, alpha: float, y: np.ndarray, abar: float = 1.0) -> np.ndarray:
    """z = C_alpha^{-1} y, the block alpha-circulant preconditioner itself (eqs.
    (1.5)-(1.7), from the prior work the paper builds on): the three steps of Section
    2.3 taken once, with the eigenvalues inverted instead of their inverse square roots:
      Step 1: DST in space, D in time, DFT in time;
      Step 2: multiply by mu^{-1};
      Step 3: inverse DFT in time, D^{-1} in time, DST in space.
    C_alpha is real, so the result is real up to rounding (asserted)."""
    d = time_scaling(g.nt, alpha)
    mu = mu_table(g, alpha, abar)
    v = dst_space(np.asarray(y, dtype=np.float64), g)
    v = _time_axis_scale(v, d).astype(np.complex128)
    v = sfft.fft(v, axis=0, workers=-1)
    v = v / mu
    v = sfft.ifft(v, axis=0, workers=-1)
    v = _time_axis_scale(v, 1.0 / d)
    z = dst_space(v.real, g) + 1j * dst_space(v.imag, g)
    scale = max(np.max(np.abs(z.real)), 1e-300)
    if np.max(np.abs(z.imag)) > 1e-9 * scale:
        raise AssertionError("C_alpha^{-1} y has a large imaginary part")
    return z.real.copy()
