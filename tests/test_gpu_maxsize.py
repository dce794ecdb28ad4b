"""GPU at the largest grids the library accepts: 1D nx = 4095 with nt = 1024, and 2D
511^2 with nt = 1024 (267 million unknowns).  The 1D case is compared with the oracle
outright (operators and the whole solve); the 2D case through its matvec and through
the explicit residual of a converged FP32-preconditioned solve under the oracle's
operator (a property that holds at any size)."""
import numpy as np
import pytest
import torch

from oracle.discretization import Grid, L_matrix
from oracle import allatonce as aao
from oracle import preconditioner as pc
from oracle import minres as mr
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _plan(nx, ny, nt, alpha=1e-3, prec="fp64"):
    from paper_2306_03574_amd import Plan
    print(f"[case] nx={nx} ny={ny} nt={nt} alpha={alpha} prec={prec}", flush=True)
    return Plan(nx, ny, nt, T=1.0, alpha=alpha, prec=prec, device=DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_largest_1d_grid_matches_oracle():
    nx, nt, alpha = 4095, 1024, 1e-2
    g = Grid(nx, 0, nt)
    src, psi0, psi1 = synth.random_source(nx, 0, nt, seed=91)
    f = aao.build_rhs(g, src, psi0, psi1)
    L = L_matrix(g)
    p = _plan(nx, 0, nt, alpha=alpha)
    fd = torch.from_numpy(f[None]).to(DEV)
    assert _rel(_host(p.apply_A(fd))[0], aao.apply_A(g, f, L)) < 1e-14
    assert _rel(_host(p.apply_Pinv(fd))[0], pc.apply_Pinv(g, alpha, f)) < 1e-11
    p32 = _plan(nx, 0, nt, alpha=alpha, prec="fp32")
    err32 = _rel(_host(p32.apply_Pinv(fd))[0], pc.apply_Pinv(g, alpha, f))
    print(f"[obs] fp32 4095x0x1024 alpha={alpha} P^-1 rel.err {err32:.3e}", flush=True)
    # twice the bound of the small shapes (3e-6 + 2e-8 / alpha): the x and time FFTs of
    # lengths 8192 and 1024 have about twice as many rounding stages
    assert err32 < 2 * (3e-6 + 2e-8 / alpha)
    u, iters, relres, status = p.solve(fd, tol=1e-8, maxit=300)
    ref = mr.minres(lambda v: aao.apply_A(g, v, L), lambda y: pc.apply_Pinv(g, alpha, y), aao.reverse_time(f),
                    tol=1e-8, maxit=300)
    assert status == [0] and iters[0] == ref.iters
    assert _rel(_host(u)[0], ref.x) < 1e-10


def test_largest_2d_grid_converges_under_the_oracle_operator():
    nx, nt, alpha = 511, 1024, 1e-3
    g = Grid(nx, nx, nt)
    rng = np.random.default_rng(92)
    src = rng.standard_normal(g.shape)
    z = np.zeros(g.level_shape)
    p = _plan(nx, nx, nt, alpha=alpha, prec="fp32")
    f = p.build_rhs(torch.from_numpy(src[None]).to(DEV), torch.from_numpy(z[None]).to(DEV),
                    torch.from_numpy(z[None]).to(DEV))
    fh = _host(f)[0]
    del src
    L = L_matrix(g)
    x = np.random.default_rng(93).standard_normal(g.shape)
    assert _rel(_host(p.apply_A(torch.from_numpy(x[None]).to(DEV)))[0], aao.apply_A(g, x, L)) < 1e-14
    del x
    u, iters, relres, status = p.solve(f, tol=1e-8, maxit=100)
    uh = _host(u)[0]
    del u
    assert status == [0]
    host_res = np.linalg.norm(fh - aao.apply_T(g, uh, L)) / np.linalg.norm(fh)
    assert host_res <= 1e-8 * (1 + 1e-6) and abs(host_res - relres[0]) <= 1e-11
