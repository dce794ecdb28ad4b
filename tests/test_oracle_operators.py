"""Pins of the oracle's operators (CPU only): the all-at-once matrix of eq. (1.2),
its symmetrisation (eqs. (1.3)-(1.4)), the right-hand side, and exact discrete
solutions (closed forms, time stepping, Table 2 of Section 3)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.discretization import (Grid, laplacian, L_matrix, L_eigenvalues, dst_space,
                                   dst_matrix, neg_laplacian_eigenvalues)
from oracle import allatonce as aao
from oracle import examples as ex
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "section3_tables.json")))

GRIDS = [(7, 0, 8), (5, 4, 6), (4, 6, 5), (15, 0, 9)]


@pytest.mark.parametrize("nx,ny,nt", GRIDS)
def test_YT_is_symmetric(nx, ny, nt):
    g = Grid(nx, ny, nt)
    A = (aao.assemble_Y(g) @ aao.assemble_T(g)).toarray()
    assert np.array_equal(A, A.T)


@pytest.mark.parametrize("nx,ny,nt", GRIDS)
def test_T_block_structure(nx, ny, nt):
    """Blocks of eq. (1.2): L on the diagonal, -2I on the first and L on the second
    block subdiagonal, zero elsewhere (checked block by block)."""
    g = Grid(nx, ny, nt)
    T = aao.assemble_T(g).toarray()
    L = L_matrix(g).toarray()
    m = g.m
    for i in range(nt):
        for j in range(nt):
            blk = T[i * m:(i + 1) * m, j * m:(j + 1) * m]
            want = L if i == j else (-2 * np.eye(m) if i == j + 1 else (L if i == j + 2 else 0 * L))
            assert np.array_equal(blk, want)


@pytest.mark.parametrize("nx,ny,nt", GRIDS)
def test_matrix_free_apply_matches_assembly(nx, ny, nt):
    g = Grid(nx, ny, nt, T=0.7)
    u = np.random.default_rng(1).standard_normal(g.shape)
    T = aao.assemble_T(g)
    Y = aao.assemble_Y(g)
    np.testing.assert_allclose(aao.apply_T(g, u).reshape(-1), T @ u.reshape(-1), rtol=0, atol=1e-12)
    np.testing.assert_allclose(aao.apply_A(g, u).reshape(-1), Y @ (T @ u.reshape(-1)), rtol=0, atol=1e-12)


@pytest.mark.parametrize("nx,ny", [(9, 0), (6, 5), (7, 7)])
def test_sine_basis_diagonalises_laplacian(nx, ny):
    """S (-Delta_h) S = diag(kappa): closed-form eigenvalues and the DST-I library
    routine against a dense symmetric eigensolver."""
    g = Grid(nx, ny, 4)
    Lap = laplacian(g).toarray()
    ev = np.sort(np.linalg.eigvalsh(-Lap))
    np.testing.assert_allclose(ev, np.sort(neg_laplacian_eigenvalues(g).reshape(-1)), rtol=1e-12)
    # S as a dense matrix (Kronecker in 2D), compared with the library DST
    S = dst_matrix(nx) if not ny else np.kron(dst_matrix(ny), dst_matrix(nx))
    np.testing.assert_allclose(S @ S, np.eye(g.m), atol=1e-13)
    D = S @ (-Lap) @ S
    np.testing.assert_allclose(np.diag(D), neg_laplacian_eigenvalues(g).reshape(-1), rtol=1e-12)
    assert np.max(np.abs(D - np.diag(np.diag(D)))) < 1e-9
    v = np.random.default_rng(2).standard_normal((3,) + g.level_shape)
    np.testing.assert_allclose(dst_space(v, g).reshape(3, -1), v.reshape(3, -1) @ S.T, atol=1e-13)
    np.testing.assert_allclose(L_eigenvalues(g), 1 + 0.5 * g.tau ** 2 * neg_laplacian_eigenvalues(g))


@pytest.mark.parametrize("nx,ny,nt", GRIDS)
def test_time_stepping_solves_T(nx, ny, nt):
    g = Grid(nx, ny, nt)
    f = np.random.default_rng(3).standard_normal(g.shape)
    u = aao.solve_time_stepping(g, f)
    u2 = spla.spsolve(aao.assemble_T(g).tocsc(), f.reshape(-1))
    np.testing.assert_allclose(u.reshape(-1), u2, rtol=1e-11, atol=1e-12)


def test_closed_form_single_mode_1d():
    """u = sin(pi x) sin(pi t), f = 0: the discrete solution is a single sine mode
    with amplitude A sin(k phi), lambda = 1 + 2 (tau/h)^2 sin^2(pi h/2),
    cos(phi) = 1/lambda, A = tau pi / (lambda sin phi).  Pins the first RHS row
    (tau psi_1) and the stencil."""
    nx, nt = 63, 64
    g = Grid(nx, 0, nt)
    src, psi0, psi1, _ = synth.manufactured_1d(nx, nt)
    f = aao.build_rhs(g, src, psi0, psi1)
    lam = 1 + 2 * (g.tau / g.hx) ** 2 * np.sin(np.pi * g.hx / 2) ** 2
    phi = np.arccos(1 / lam)
    A = g.tau * np.pi / (lam * np.sin(phi))
    k = np.arange(1, nt + 1)
    (x,) = g.points()
    u_cf = A * np.sin(k * phi)[:, None] * np.sin(np.pi * x)[None, :]
    np.testing.assert_allclose(aao.apply_T(g, u_cf), f, atol=1e-14)
    np.testing.assert_allclose(aao.solve_time_stepping(g, f), u_cf, atol=1e-13)


def test_closed_form_single_mode_2d():
    """u = sin(pi x) sin(pi y) sin(pi t): the mode amplitude obeys the scalar
    recurrence lambda a1 = tau pi, lambda a2 - 2 a1 = tau^2 pi^2 sin(pi tau),
    lambda a_k - 2 a_{k-1} + lambda a_{k-2} = tau^2 pi^2 sin((k-1) pi tau)."""
    n, nt = 31, 32
    g = Grid(n, n, nt)
    src, psi0, psi1, _ = synth.manufactured_2d(n, n, nt)
    f = aao.build_rhs(g, src, psi0, psi1)
    lam = 1 + 4 * (g.tau / g.hx) ** 2 * np.sin(np.pi * g.hx / 2) ** 2
    a = np.zeros(nt)
    rhs = g.tau ** 2 * np.pi ** 2 * np.sin(np.arange(nt) * np.pi * g.tau)
    a[0] = g.tau * np.pi / lam
    a[1] = (rhs[1] + 2 * a[0]) / lam
    for k in range(2, nt):
        a[k] = (rhs[k] + 2 * a[k - 1] - lam * a[k - 2]) / lam
    X, Y = g.points()
    u_cf = a[:, None, None] * (np.sin(np.pi * X) * np.sin(np.pi * Y))[None]
    np.testing.assert_allclose(aao.solve_time_stepping(g, f), u_cf, atol=1e-13)


def _table2_exact(lt, lh, rhs_variant=None):
    nt, nx = 2 ** lt, 2 ** lh - 1
    g = Grid(nx, nx, nt)
    src, psi0, psi1, exact = ex.example1_data(g)
    f = aao.build_rhs(g, src, psi0, psi1)
    if rhs_variant == "tau_L_psi1":
        L = L_matrix(g)
        f[0] += g.tau * ((L @ psi1.reshape(-1)).reshape(psi1.shape) - psi1)
    u = aao.solve_time_stepping(g, f)
    return ex.error_E(g, u, exact)


@pytest.mark.parametrize("row", [r for r in GOLD["table2"]["rows"] if r[1] <= 5])
def test_table2_exact_discrete_error(row):
    """Table 2's P_1 column equals the error of the exact discrete solution (MINRES
    converged); reproduced to the printed three digits."""
    lt, lh, _, e_p1, _ = row
    e = _table2_exact(lt, lh)
    assert abs(e - e_p1) <= 0.006 * e_p1, (e, e_p1)


def test_table2_rejects_ghost_point_rhs_reading():
    """Planted alternative reading tau L psi_1 in block 1 misses Table 2."""
    e = _table2_exact(4, 4, rhs_variant="tau_L_psi1")
    assert abs(e - 3.04e-4) > 0.1 * 3.04e-4


def test_rhs_rows():
    """Rows of f, eq. (1.2), against an independent evaluation from the definition."""
    g = Grid(5, 4, 6, T=0.9)
    rng = np.random.default_rng(4)
    src = rng.standard_normal(g.shape)
    psi0 = rng.standard_normal(g.level_shape)
    psi1 = rng.standard_normal(g.level_shape)
    f = aao.build_rhs(g, src, psi0, psi1)
    Lap = laplacian(g).toarray()
    t2 = g.tau ** 2
    np.testing.assert_allclose(f[0].reshape(-1), (t2 * src[0] / 2 + psi1 * g.tau + psi0).reshape(-1), atol=1e-14)
    Lpsi0 = psi0.reshape(-1) - 0.5 * t2 * Lap @ psi0.reshape(-1)
    np.testing.assert_allclose(f[1].reshape(-1), t2 * src[1].reshape(-1) - Lpsi0, atol=1e-13)
    np.testing.assert_allclose(f[2:], t2 * src[2:], atol=1e-15)
