"""Pins of the oracle's block alpha-circulant preconditioner C_alpha^{-1} and of its
right-preconditioned GMRES (eqs. (1.2), (1.5)-(1.7)), CPU only: a sparse direct solve
with the assembled C_alpha, the brute-force Krylov minimiser, exact termination
within rank(C_alpha - T) + 1 steps, agreement with time stepping, and restart
consistency."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.discretization import Grid
from oracle import allatonce as aao
from oracle import preconditioner as pc
from oracle import gmres as gm
import synth


@pytest.mark.parametrize("nx,ny,nt,alpha", [(9, 0, 8, 0.1), (7, 5, 8, 1e-2), (15, 7, 16, 1e-3), (6, 4, 8, 1e-6)])
def test_C_inv_matches_direct_solve(nx, ny, nt, alpha):
    g = Grid(nx, ny, nt)
    y = np.random.default_rng(nx + ny).standard_normal(g.shape)
    z = pc.apply_C_inv(g, alpha, y)
    zd = spla.spsolve(pc.assemble_C(g, alpha).tocsc(), y.reshape(-1)).reshape(g.shape)
    assert np.max(np.abs(z - zd)) <= 1e-9 * np.max(np.abs(zd))
    back = (pc.assemble_C(g, alpha) @ z.reshape(-1)).reshape(g.shape)
    assert np.max(np.abs(back - y)) <= 1e-9 * np.max(np.abs(y))


def test_planted_scaling_swap_is_detected():
    """D and D^{-1} exchanged in the apply (a plausible slip) fails the direct solve."""
    g = Grid(7, 5, 8)
    alpha = 1e-2
    y = np.random.default_rng(1).standard_normal(g.shape)
    d = pc.time_scaling(g.nt, alpha)
    mu = pc.mu_table(g, alpha)
    v = pc.dst_space(y, g) / d.reshape(-1, 1, 1)
    v = np.fft.ifft(np.fft.fft(v, axis=0) / mu, axis=0) * d.reshape(-1, 1, 1)
    wrong = pc.dst_space(v.real, g)
    zd = spla.spsolve(pc.assemble_C(g, alpha).tocsc(), y.reshape(-1)).reshape(g.shape)
    assert np.max(np.abs(wrong - zd)) > 1e-3 * np.max(np.abs(zd))


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_iterates_match_brute_force(k):
    g = Grid(5, 3, 8)
    alpha = 0.2
    src, p0, p1 = synth.random_source(5, 3, 8, seed=31)
    f = aao.build_rhs(g, src, p0, p1)
    T = aao.assemble_T(g).toarray()
    Minv = np.column_stack([pc.apply_C_inv(g, alpha, e.reshape(g.shape)).reshape(-1) for e in np.eye(g.N)])
    ref = gm.krylov_minimiser_right(T, Minv, f, k)
    res = gm.gmres(lambda u: aao.apply_T(g, u), lambda y: pc.apply_C_inv(g, alpha, y), f, fixed_iters=k, restart=50)
    assert np.max(np.abs(res.x.reshape(-1) - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_terminates_within_rank_of_the_difference():
    """C_alpha - T holds only the alpha-weighted corner blocks, all in the last two
    block columns (rank <= 2m, here exactly 2m), so T C_alpha^{-1} is the identity plus
    a rank-2m term and exact GMRES ends in at most 2m + 1 steps; in FP64 the residual
    is at rounding level by then."""
    g = Grid(5, 0, 16)
    alpha = 0.5
    diff = (aao.assemble_T(g) - pc.assemble_C(g, alpha)).toarray()
    assert np.linalg.matrix_rank(diff) == 2 * g.m
    src, p0, p1 = synth.random_source(5, 0, 16, seed=2)
    f = aao.build_rhs(g, src, p0, p1)
    res = gm.gmres(lambda u: aao.apply_T(g, u), lambda y: pc.apply_C_inv(g, alpha, y), f, tol=1e-11, maxit=200,
                   restart=200)
    assert res.converged and res.iters <= 2 * g.m + 1


def test_restart_cycle_equals_unrestarted_prefix_and_converges():
    g = Grid(15, 7, 16)
    alpha = 0.3
    src, p0, p1 = synth.random_source(15, 7, 16, seed=3)
    f = aao.build_rhs(g, src, p0, p1)
    A = lambda u: aao.apply_T(g, u)
    M = lambda y: pc.apply_C_inv(g, alpha, y)
    one = gm.gmres(A, M, f, fixed_iters=3, restart=3)
    long = gm.gmres(A, M, f, fixed_iters=3, restart=30)
    assert np.max(np.abs(one.x - long.x)) <= 1e-12 * np.max(np.abs(long.x))
    res = gm.gmres(A, M, f, tol=1e-10, maxit=300, restart=3)
    assert res.converged and res.relres <= 1e-10
    full = gm.gmres(A, M, f, tol=1e-10, maxit=300, restart=300)
    assert full.iters <= res.iters


def test_solution_matches_time_stepping():
    g = Grid(31, 15, 32)
    src, p0, p1 = synth.random_source(31, 15, 32, seed=4)
    f = aao.build_rhs(g, src, p0, p1)
    res = gm.gmres(lambda u: aao.apply_T(g, u), lambda y: pc.apply_C_inv(g, 1e-3, y), f, tol=1e-12, maxit=50)
    ref = aao.solve_time_stepping(g, f)
    assert res.converged and np.max(np.abs(res.x - ref)) <= 1e-9 * np.max(np.abs(ref))
