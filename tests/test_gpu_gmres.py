"""GPU parity of the non-symmetric path: T x in natural order, the block
alpha-circulant preconditioner C_alpha^{-1} (eqs. (1.5)-(1.7)) and right-preconditioned
restarted GMRES, through the C ABI against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle.discretization import Grid
from oracle import allatonce as aao
from oracle import preconditioner as pc
from oracle import gmres as gm
from oracle import varcoef as vc
from oracle import examples as ex
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _plan(nx, ny, nt, alpha=1e-3, prec="fp64", batch=1):
    from paper_2306_03574_amd import Plan
    print(f"[case] gmres nx={nx} ny={ny} nt={nt} alpha={alpha} prec={prec} batch={batch}", flush=True)
    return Plan(nx, ny, nt, T=1.0, alpha=alpha, prec=prec, batch=batch, device=DEV)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


SHAPES = [(7, 0, 8), (63, 0, 64), (1023, 0, 8), (7, 7, 8), (15, 7, 16), (31, 31, 32), (127, 15, 8)]


@pytest.mark.parametrize("nx,ny,nt", SHAPES)
def test_apply_T_natural_order(nx, ny, nt):
    g = Grid(nx, ny, nt)
    x = synth.random_source(nx, ny, nt, seed=21)[0]
    p = _plan(nx, ny, nt)
    y = _host(p.apply_T(_dev(x[None])))[0]
    assert _rel(y, aao.apply_T(g, x)) < 1e-14
    if ny:
        apts, axh, ayh = vc.coefficient_samples(g, lambda X, Y: 1.0 + X + Y * Y)
        p.set_coefficient(axh, ayh, float(apts.mean()))
        y = _host(p.apply_T(_dev(x[None])))[0]
        assert _rel(y, vc.apply_T_var(g, x, vc.L_var(g, axh, ayh))) < 1e-14


@pytest.mark.parametrize("nx,ny,nt,alpha", [(7, 0, 8, 1e-1), (63, 0, 64, 1e-3), (15, 7, 16, 1e-2), (31, 31, 32, 1e-3),
                                            (127, 15, 8, 0.5), (255, 0, 32, 1e-6)])
def test_apply_Cinv(nx, ny, nt, alpha):
    g = Grid(nx, ny, nt)
    r = synth.random_source(nx, ny, nt, seed=22)[0]
    ref = pc.apply_C_inv(g, alpha, r)
    z = _host(_plan(nx, ny, nt, alpha=alpha).apply_Cinv(_dev(r[None])))[0]
    assert _rel(z, ref) < 1e-11 * max(1.0, 1e-3 / alpha)
    z32 = _host(_plan(nx, ny, nt, alpha=alpha, prec="fp32").apply_Cinv(_dev(r[None])))[0]
    # FP32 transforms: rounding amplified by up to 1/alpha by the D_alpha^{-1} scaling
    # (the bound of the FP32 P^{-1} test)
    err = _rel(z32, ref)
    print(f"[obs] fp32 C_alpha^-1 alpha={alpha} rel.err {err:.3e}", flush=True)
    # measured 2.5e-7 (alpha 0.1, 0.5), 8.4e-7 (1e-2), 4.7e-6 .. 6.7e-6 (1e-3), 1.8e-3 (1e-6)
    assert err < 3e-6 + 2e-8 / alpha
    zn = _host(_plan(nx, ny, nt, alpha=alpha, prec="none").apply_Cinv(_dev(r[None])))[0]
    assert np.array_equal(zn, r)


@pytest.mark.parametrize("k,restart", [(1, 15), (2, 15), (5, 15), (7, 3), (9, 2)])
def test_fixed_iterates_match_oracle(k, restart):
    """The iterate after k steps (restarts included) equals the oracle's."""
    nx, ny, nt, alpha = 15, 7, 16, 0.3
    g = Grid(nx, ny, nt)
    src, p0, p1 = synth.random_source(nx, ny, nt, seed=23)
    f = aao.build_rhs(g, src, p0, p1)
    ref = gm.gmres(lambda u: aao.apply_T(g, u), lambda y: pc.apply_C_inv(g, alpha, y), f, fixed_iters=k,
                   restart=restart)
    p = _plan(nx, ny, nt, alpha=alpha)
    u, iters, relres, status = p.gmres(_dev(f[None]), tol=1e-30, maxit=k, restart=restart)
    assert iters == [k] and status == [-4]
    assert _rel(_host(u)[0], ref.x) < 1e-10
    assert abs(relres[0] - ref.relres) <= 1e-9 * ref.relres


@pytest.mark.parametrize("nx,ny,nt,alpha,restart", [(31, 15, 32, 1e-3, 15), (63, 0, 64, 1e-1, 15),
                                                    (63, 0, 64, 1e-1, 2), (31, 31, 32, 1e-2, 4)])
def test_solve_matches_oracle_and_time_stepping(nx, ny, nt, alpha, restart):
    g = Grid(nx, ny, nt)
    src, p0, p1 = synth.random_source(nx, ny, nt, seed=24)
    f = aao.build_rhs(g, src, p0, p1)
    ref = gm.gmres(lambda u: aao.apply_T(g, u), lambda y: pc.apply_C_inv(g, alpha, y), f, tol=1e-10, maxit=300,
                   restart=restart)
    p = _plan(nx, ny, nt, alpha=alpha)
    u, iters, relres, status = p.gmres(_dev(f[None]), tol=1e-10, maxit=300, restart=restart)
    assert status == [0] and relres[0] <= 1e-10
    assert abs(iters[0] - ref.iters) <= 1, (iters[0], ref.iters)
    exact = aao.solve_time_stepping(g, f)
    assert _rel(_host(u)[0], exact) < 1e-7


def test_example1_two_steps_at_small_alpha():
    """At alpha = 1e-6, C_alpha is T up to the corner blocks, so GMRES needs about as
    few steps as MINRES-P_alpha (2 in Table 1); the error matches Table 2's."""
    g = Grid(15, 15, 16)
    src, psi0, psi1, exact = ex.example1_data(g)
    p = _plan(15, 15, 16, alpha=1e-6)
    f = p.build_rhs(_dev(src[None]), _dev(psi0[None]), _dev(psi1[None]))
    fh = _host(f)[0]
    ref = gm.gmres(lambda u: aao.apply_T(g, u), lambda y: pc.apply_C_inv(g, 1e-6, y), fh, tol=1e-6, maxit=50)
    u, iters, relres, status = p.gmres(f, tol=1e-6, maxit=50)
    assert status == [0] and iters[0] == ref.iters <= 3
    assert abs(ex.error_E(g, _host(u)[0], exact) - 0.000304) <= 0.006 * 0.000304


def test_batch_equals_solo_and_zero_rhs():
    nx, ny, nt, B = 31, 15, 16, 3
    g = Grid(nx, ny, nt)
    fs = []
    for b in range(B):
        src, p0, p1 = synth.random_source(nx, ny, nt, seed=50 + b)
        fs.append(aao.build_rhs(g, src, p0, p1))
    fs[1] = np.zeros_like(fs[1])
    pb = _plan(nx, ny, nt, alpha=0.05, batch=B)
    ub, itb, rrb, stb = pb.gmres(_dev(np.stack(fs)), tol=1e-9, maxit=100, restart=4)
    assert stb == [0, 0, 0] and itb[1] == 0 and not torch.any(ub[1])
    for b in (0, 2):
        ps = _plan(nx, ny, nt, alpha=0.05)
        us, its, rrs, sts = ps.gmres(_dev(fs[b][None]), tol=1e-9, maxit=100, restart=4)
        assert its[0] == itb[b] and rrs[0] == rrb[b] and torch.equal(us[0], ub[b])


def test_bad_arguments():
    from paper_2306_03574_amd.abac import AbacError
    p = _plan(15, 7, 16)
    f = p.empty()
    f.zero_()
    for kw in (dict(restart=0), dict(restart=16), dict(maxit=0), dict(tol=0.0)):
        with pytest.raises(AbacError):
            p.gmres(f, **kw)
