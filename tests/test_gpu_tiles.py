"""Every legal tile of the tuned transform passes, run through the oracle comparison.

The plan's tuner times every legal workgroup size of the first x-DST pass, the y-DST
pass and the time pass and keeps the fastest, so the tile a benchmark run executes is
decided by timing.  Here each legal tile of each pass is forced (abac_plan_set_tiles)
at every transform length the workloads use:

* first and last x-DST lengths 2(nx+1): 256 (the FP64 127^2 batch), 512 (255, 255^2), 1024 (511^2),
  2048 (1D 1023), 8192 (1D 4095);
* y-DST lengths 2(ny+1): 256, 512, 1024;
* time lengths nt: 64, 128, 256, 512, 1024.

For each tile: P_alpha^{-1} r against the FP64 oracle (FP64 transforms: 1e-10, the bar
of the FP64 path; the D_alpha^{-1} scaling amplifies rounding by up to 1/alpha and at
nt = 1024 the two FP64 routes differ by 4e-11; FP32 transforms: the FP32 bound), bitwise equality with the plan's tuned
tile (the arithmetic per sequence is the same, and the time pass sums its partials of
<q, P^{-1} q> in an order fixed by the sequence length), and
the Lanczos path of the first pass through a fixed number of MINRES iterations, whose
iterate is bitwise equal to the tuned tile's and (FP64) within 1e-10 of the oracle's.
The grids are small in the dimensions the pass does not transform.
"""
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
CANDIDATES = [64, 128, 256, 512, 1024]
ALPHA = 1e-3
K_FIXED = 3


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _grid_for(kind, L):
    """A small grid whose pass `kind` has transform length L (separate x and y passes)."""
    if kind in ("dstx_fwd", "dstx_inv"):
        nx = L // 2 - 1
        return (nx, 0, 8) if L > 1024 else (nx, 7, 8)
    if kind == "dsty":
        return (7, L // 2 - 1, 8)
    return (15, 7, L)


CASES = ([(k, L) for k in ("dstx_fwd", "dstx_inv") for L in (256, 512, 1024, 2048, 8192)] +
         [("dsty", L) for L in (256, 512, 1024)] + [("time", L) for L in (64, 128, 256, 512, 1024)])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,L", CASES)
def test_every_legal_tile_matches_oracle(kind, L, prec):
    from paper_2306_03574_amd import Plan
    from paper_2306_03574_amd.abac import AbacError, EINVAL
    nx, ny, nt = _grid_for(kind, L)
    g = Grid(nx, ny, nt)
    _say(f"tiles {kind} L={L} prec={prec} grid nx={nx} ny={ny} nt={nt}")
    p = Plan(nx, ny, nt, alpha=ALPHA, prec=prec, device=DEV)
    tiles = p.tiles()
    assert tiles["slab"] == 0 and tiles["small"] == 0, tiles
    tuned = tiles[kind]
    r = np.random.default_rng(31).standard_normal(g.shape)
    src, psi0, psi1 = synth.random_source(nx, ny, nt, seed=32)
    f = aao.build_rhs(g, src, psi0, psi1)
    ref_z = pc.apply_Pinv(g, ALPHA, r)
    Lm = L_matrix(g)
    ref_x = mr.minres(lambda u: aao.apply_A(g, u, Lm), lambda y: pc.apply_Pinv(g, ALPHA, y),
                      aao.reverse_time(f), fixed_iters=K_FIXED).x
    zbound = 1e-10 if prec == "fp64" else 7e-5   # FP32: measured 5e-6 .. 1.4e-5 (about eps32 / (5 alpha)), times 5

    def run():
        z = _host(p.apply_Pinv(_dev(r[None])))[0]
        u, iters, _, _ = p.solve(_dev(f[None]), tol=1e-30, maxit=K_FIXED)
        assert iters == [K_FIXED]
        return z, _host(u)[0]

    _say(f"tiles {kind} L={L} prec={prec} tuned wg={tuned}")
    z0, u0 = run()
    print(f"[obs] tiles {kind} L={L} prec={prec} P^-1 rel.err {_rel(z0, ref_z):.3e}", flush=True)
    assert _rel(z0, ref_z) < zbound
    if prec == "fp64":
        assert _rel(u0, ref_x) < 1e-10
    legal = []
    for wg in CANDIDATES:
        try:
            p.set_tiles(**{kind: wg})
        except AbacError as e:
            assert e.status == EINVAL
            continue
        legal.append(wg)
        _say(f"tiles {kind} L={L} prec={prec} wg={wg}")
        z, u = run()
        assert np.array_equal(z, z0), (kind, L, prec, wg, _rel(z, z0))
        assert np.array_equal(u, u0), (kind, L, prec, wg, _rel(u, u0))
        assert _rel(z, ref_z) < zbound
    assert tuned in legal, (tuned, legal)
