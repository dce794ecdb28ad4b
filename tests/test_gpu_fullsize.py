"""GPU parity at the benchmark workloads' full sizes, in the launch configuration the
benchmark times: the same plan shape, batch and preconditioner precision, the same
seeded inputs (the benchmark's own input recipe), right-hand sides assembled on the
GPU and solved to tol 1e-8 with the graph-replayed iteration.

Where the FP64 CPU oracle finishes in seconds to a minute at these sizes it computes
the whole result: the operators of the 255^2 x 256 and 511^2 x 512 grids, the whole
MINRES solve of the 255^2 x 256 workload (at alpha 1e-3 and 1e-2, and its twin with an
i.i.d. random source) and of sampled right-hand sides of the 64 x 127^2 x 128 batch.  The 511^2 x 512 solve (about two minutes for the oracle) is
checked through properties that hold at any size: the explicit residual of the
returned iterate under the oracle's operator, and the iteration count against the
FP64-preconditioned solve of the same system.

Each workload builds its inputs once (module fixtures); every case prints its
identity before touching the GPU.
"""
import numpy as np
import pytest
import torch

import bench
from oracle.discretization import Grid, L_matrix
from oracle import allatonce as aao
from oracle import preconditioner as pc
from oracle import minres as mr

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-8


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _plan(w, prec, alpha=None):
    from paper_2306_03574_amd import Plan
    alpha = w["alpha"] if alpha is None else alpha
    _say(f"plan nx={w['nx']} ny={w['ny']} nt={w['nt']} alpha={alpha} batch={w['batch']} prec={prec}")
    return Plan(w["nx"], w["ny"], w["nt"], T=1.0, alpha=alpha, prec=prec, batch=w["batch"], device=DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


class _Workload:
    def __init__(self, name):
        self.name = name
        self.w = bench.WORKLOADS[name]
        self.g = Grid(self.w["nx"], self.w["ny"], self.w["nt"], T=1.0)
        _say(f"inputs {name}")
        self.src, self.p0, self.p1 = bench.make_inputs(self.w)
        self._L = None

    @property
    def L(self):
        if self._L is None:
            self._L = L_matrix(self.g)
        return self._L

    def device_inputs(self):
        return (torch.from_numpy(self.src).to(DEV), torch.from_numpy(self.p0).to(DEV),
                torch.from_numpy(self.p1).to(DEV))

    def rhs(self, b):
        return aao.build_rhs(self.g, self.src[b], self.p0[b], self.p1[b])

    def gpu_solve(self, prec, alpha=None):
        p = _plan(self.w, prec, alpha)
        d = self.device_inputs()
        f = p.build_rhs(*d)
        u, iters, relres, status = p.solve(f, tol=TOL, maxit=500)
        return p, _host(f), _host(u), iters, relres, status


@pytest.fixture(scope="module")
def c2():
    return _Workload("wave2d_255x255x256")


@pytest.fixture(scope="module")
def c2r():
    return _Workload("wave2d_255x255x256_random")


@pytest.fixture(scope="module")
def c3():
    return _Workload("wave2d_511x511x512")


@pytest.fixture(scope="module")
def c4():
    return _Workload("batch64_wave2d_127x127x128")


# --- 255^2 x 256, FP64 end to end ---------------------------------------------------

def test_c2_operators(c2):
    """RHS assembly, Y T and P_alpha^{-1} on the full grid against the oracle."""
    p = _plan(c2.w, "fp64")
    f = p.build_rhs(*c2.device_inputs())
    fh = _host(f)[0]
    assert _rel(fh, c2.rhs(0)) < 1e-14
    x = np.random.default_rng(81).standard_normal(c2.g.shape)
    xd = torch.from_numpy(x[None]).to(DEV)
    _say("c2 apply_A")
    assert _rel(_host(p.apply_A(xd))[0], aao.apply_A(c2.g, x, c2.L)) < 1e-14
    _say("c2 apply_Pinv")
    assert _rel(_host(p.apply_Pinv(xd))[0], pc.apply_Pinv(c2.g, c2.w["alpha"], x)) < 1e-11


def _whole_solve_matches_oracle(wl, alpha):
    _, fh, uh, iters, relres, status = wl.gpu_solve("fp64", alpha)
    f = fh[0]
    _say(f"{wl.name} oracle solve alpha={alpha}")
    ref = mr.minres(lambda v: aao.apply_A(wl.g, v, wl.L), lambda y: pc.apply_Pinv(wl.g, alpha, y),
                    aao.reverse_time(f), tol=TOL, maxit=500)
    assert status == [0] and ref.converged
    assert iters[0] == ref.iters
    assert _rel(uh[0], ref.x) < 1e-10
    host_res = np.linalg.norm(f - aao.apply_T(wl.g, uh[0], wl.L)) / np.linalg.norm(f)
    assert host_res <= TOL and abs(host_res - relres[0]) <= 1e-3 * TOL
    return iters[0]


def test_c2_solve_matches_oracle(c2):
    """The whole solve: same iteration count, iterate within 1e-10, explicit residual."""
    _whole_solve_matches_oracle(c2, c2.w["alpha"])


def test_c2_alpha_1e2_solve_matches_oracle(c2):
    """The same grid and source at the workload's other alpha, 1e-2."""
    _whole_solve_matches_oracle(c2, 1e-2)


def test_c2_random_source_twin_matches_oracle(c2r):
    """The grid with an i.i.d. N(0,1) source (seed 2): a right-hand side without the
    manufactured solution's smoothness, solved to the same bar."""
    assert c2r.w["source"] == "random" and c2r.w["seed"] == 2
    _whole_solve_matches_oracle(c2r, c2r.w["alpha"])


# --- 64 x 127^2 x 128 batch --------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c4_batch_solve(c4, prec):
    """Every right-hand side of the batch converges under the oracle's operator; with the
    FP64 preconditioner sampled right-hand sides match the oracle's solve (count and
    iterate), with FP32 transforms their counts stay within 2 of the oracle's."""
    _, fh, uh, iters, relres, status = c4.gpu_solve(prec)
    B = c4.w["batch"]
    assert status == [0] * B
    for b in range(B):
        host_res = np.linalg.norm(fh[b] - aao.apply_T(c4.g, uh[b], c4.L)) / np.linalg.norm(fh[b])
        assert host_res <= TOL * (1 + 1e-6), (b, host_res)
    for b in (0, 37, B - 1):
        assert np.array_equal(fh[b], c4.rhs(b)) or _rel(fh[b], c4.rhs(b)) < 1e-14
        _say(f"c4 oracle solve rhs {b}")
        ref = mr.minres(lambda v: aao.apply_A(c4.g, v, c4.L), lambda y: pc.apply_Pinv(c4.g, c4.w["alpha"], y),
                        aao.reverse_time(fh[b]), tol=TOL, maxit=500)
        if prec == "fp64":
            assert iters[b] == ref.iters
            assert _rel(uh[b], ref.x) < 1e-10
        else:
            assert abs(iters[b] - ref.iters) <= 2, (iters[b], ref.iters)


# --- 511^2 x 512, FP32 transforms --------------------------------------------------

def test_c3_operators(c3):
    """RHS assembly and Y T to rounding; the FP32-transform P_alpha^{-1} within its
    error level eps32 / alpha of the FP64 oracle."""
    p = _plan(c3.w, "fp32")
    f = p.build_rhs(*c3.device_inputs())
    fh = _host(f)[0]
    del f
    assert _rel(fh, c3.rhs(0)) < 1e-14
    fd = torch.from_numpy(fh[None]).to(DEV)
    _say("c3 apply_A")
    assert _rel(_host(p.apply_A(fd))[0], aao.apply_A(c3.g, fh, c3.L)) < 1e-14
    _say("c3 apply_Pinv")
    z = _host(p.apply_Pinv(fd))[0]
    assert _rel(z, pc.apply_Pinv(c3.g, c3.w["alpha"], fh)) < 50 * 6e-8 / c3.w["alpha"]


def test_c3_solve_properties(c3):
    """FP32-transform solve: converged under the oracle's operator, and within two
    iterations of the FP64-preconditioned solve of the same system."""
    _, fh, uh, iters, relres, status = c3.gpu_solve("fp32")
    f = fh[0]
    assert status == [0]
    _say("c3 host residual")
    host_res = np.linalg.norm(f - aao.apply_T(c3.g, uh[0], c3.L)) / np.linalg.norm(f)
    assert host_res <= TOL * (1 + 1e-6) and abs(host_res - relres[0]) <= 1e-3 * TOL
    del uh
    _, _, _, iters64, _, status64 = c3.gpu_solve("fp64")
    assert status64 == [0]
    assert abs(iters[0] - iters64[0]) <= 2, (iters[0], iters64[0])
