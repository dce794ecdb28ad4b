"""Pins of the oracle's ABAC preconditioner (CPU only): eigenvalues of C_alpha
(eq. (1.7), Appendix A), the principal square root (eq. (1.8)), the lemmas of
Section 2 as invariants on tiny sizes, and the fast apply of Section 2.3 against the
dense definition (eq. (1.9))."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.optimize import linear_sum_assignment

from oracle.discretization import Grid, L_matrix, L_eigenvalues
from oracle import allatonce as aao
from oracle import preconditioner as pc

TINY = [(5, 0, 6, 0.1), (3, 4, 6, 1e-2), (4, 3, 5, 0.3), (7, 0, 8, 1e-3), (4, 4, 4, 0.5)]


def _match(ev, mu):
    D = np.abs(ev[:, None] - mu[None, :])
    r, c = linear_sum_assignment(D)
    return np.max(D[r, c])


@pytest.mark.parametrize("nx,ny,nt,alpha", TINY)
def test_eigenvalues_of_C_alpha(nx, ny, nt, alpha):
    """eig(C_alpha) = {lambda_j(L) lambda_{1,k} + lambda_{2,k}} (eq. (1.7)); the
    reading with -2 counted twice (Lambda_{alpha,2} (x) (-2 I)) is rejected."""
    g = Grid(nx, ny, nt)
    ev = np.linalg.eigvals(pc.assemble_C(g, alpha).toarray())
    mu = pc.mu_table(g, alpha).reshape(-1)
    assert _match(ev, mu) < 1e-11 * np.max(np.abs(mu))
    l1, l2 = pc.time_eigenvalues(nt, alpha)
    lam = L_eigenvalues(g).reshape(-1)
    wrong = (lam[None, :] * l1[:, None] - 2 * l2[:, None]).reshape(-1)
    assert _match(ev, wrong) > 0.1


@pytest.mark.parametrize("nx,ny,nt,alpha", TINY)
def test_spectrum_avoids_negative_axis(nx, ny, nt, alpha):
    """Lemma on C_alpha in Section 2.1 (proof in Appendix A): no eigenvalue on (-inf, 0]."""
    g = Grid(nx, ny, nt)
    mu = pc.mu_table(g, alpha)
    assert np.all((mu.real > 0) | (np.abs(mu.imag) > 1e-12))


@pytest.mark.parametrize("nx,ny,nt,alpha", TINY)
def test_sqrt_lemmas(nx, ny, nt, alpha):
    """Lemma on C_alpha^{1/2} (Section 2.1): real, Y C^{1/2} symmetric; hence
    (C^{-1/2})^T = Y C^{-1/2} Y; P_alpha symmetric positive definite (eq. (1.9))."""
    g = Grid(nx, ny, nt)
    S = pc.dense_sqrt_C(g, alpha)
    C = pc.assemble_C(g, alpha).toarray()
    np.testing.assert_allclose(S @ S, C, atol=1e-10 * np.max(np.abs(C)))
    Y = aao.assemble_Y(g).toarray()
    YS = Y @ S
    assert np.max(np.abs(YS - YS.T)) < 1e-10 * np.max(np.abs(S))
    Sinv = np.linalg.inv(S)
    assert np.max(np.abs(Sinv.T - Y @ Sinv @ Y)) < 1e-9 * np.max(np.abs(Sinv))
    P = S.T @ S
    assert np.min(np.linalg.eigvalsh(0.5 * (P + P.T))) > 0
    # eigenvalues of C^{1/2} in the open right half plane (principal branch)
    assert np.min(np.linalg.eigvals(S).real) > 0


@pytest.mark.parametrize("nx,ny,nt,alpha", TINY + [(6, 0, 16, 1e-6)])
def test_fast_apply_matches_dense(nx, ny, nt, alpha):
    """Section 2.3 (three steps, twice) == dense P_alpha^{-1} y."""
    g = Grid(nx, ny, nt, T=1.3)
    y = np.random.default_rng(5).standard_normal(g.shape)
    zd = pc.dense_apply_Pinv(g, alpha, y)
    zm = pc.apply_Pinv(g, alpha, y)
    tol = 1e-12 if alpha >= 1e-3 else 1e-8
    assert np.max(np.abs(zd - zm)) <= tol * np.max(np.abs(zd))


def test_transposed_factor_order_is_detected():
    """Planted mistake: (C^{-1/2})^T C^{-1/2} y instead of C^{-1/2} (C^{-1/2})^T y."""
    g = Grid(4, 3, 6)
    alpha = 0.05
    y = np.random.default_rng(6).standard_normal(g.shape)
    zd = pc.dense_apply_Pinv(g, alpha, y)
    wrong = pc.apply_C_inv_sqrt_T(g, alpha, pc.apply_C_inv_sqrt(g, alpha, y).real).real
    assert np.max(np.abs(zd - wrong)) > 1e-3 * np.max(np.abs(zd))


@pytest.mark.parametrize("nx,ny,nt,alpha", [(5, 0, 6, 0.1), (3, 3, 6, 0.02), (6, 0, 8, 0.3)])
def test_Q_orthogonal_and_spectrum_bound(nx, ny, nt, alpha):
    """Section 2.2: Q = P^{-1/2} Y C P^{-1/2} is symmetric orthogonal; the spectrum of
    P^{-1} Y T lies in [-1-e, -1+e] U [1-e, 1+e], e = ||P^{-1/2} Y R P^{-1/2}||_2,
    and ||R_alpha||_2 = alpha (sqrt(||L||^2 + 1) + 1)."""
    g = Grid(nx, ny, nt)
    P = pc.dense_P(g, alpha)
    w, V = np.linalg.eigh(0.5 * (P + P.T))
    Pmh = V @ np.diag(w ** -0.5) @ V.T
    Y = aao.assemble_Y(g).toarray()
    C = pc.assemble_C(g, alpha).toarray()
    T = aao.assemble_T(g).toarray()
    Q = Pmh @ Y @ C @ Pmh
    assert np.max(np.abs(Q - Q.T)) < 1e-9
    assert np.max(np.abs(Q @ Q.T - np.eye(g.N))) < 1e-9
    R = C - T
    E = Pmh @ Y @ R @ Pmh
    e = np.linalg.norm(E, 2)
    ev = np.linalg.eigvals(np.linalg.solve(P, Y @ T)).real
    assert np.all(np.minimum(np.abs(ev - 1), np.abs(ev + 1)) <= e + 1e-9)
    Lnorm = np.linalg.norm(L_matrix(g).toarray(), 2)
    assert abs(np.linalg.norm(R, 2) - alpha * (np.sqrt(Lnorm ** 2 + 1) + 1)) < 1e-10


def test_ideal_preconditioner_two_eigenvalues():
    """Proposition on the ideal preconditioner (Section 2.1): with
    (T^{1/2})^T T^{1/2} the preconditioned spectrum is exactly {-1, +1}."""
    g = Grid(4, 3, 5)
    T = aao.assemble_T(g).toarray()
    S = np.real(sla.sqrtm(T))
    Y = aao.assemble_Y(g).toarray()
    ev = np.linalg.eigvals(np.linalg.solve(S.T @ S, Y @ T))
    assert np.max(np.minimum(np.abs(ev - 1), np.abs(ev + 1))) < 1e-8


def test_alpha_one_is_polar_factor():
    """Remark after eq. (1.10): at alpha = 1, P_1 = |C_1| = sqrt(C_1^T C_1), the
    symmetric factor of the polar decomposition (library routine)."""
    g = Grid(4, 0, 6)
    C1 = pc.assemble_C(g, 1.0).toarray()
    _, H = sla.polar(C1)
    P1 = pc.dense_P(g, 1.0)
    np.testing.assert_allclose(P1, H, atol=1e-9)
    y = np.random.default_rng(7).standard_normal(g.shape)
    z = pc.apply_Pinv(g, 1.0, y)
    np.testing.assert_allclose(z.reshape(-1), np.linalg.solve(H, y.reshape(-1)), atol=1e-9)
