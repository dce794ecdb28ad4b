"""Solves of different grids advanced together (abac_group_*): one launch per MINRES step
for every member.  Each member's iterate, iteration count and residual must be bitwise
those of the same plan's own solve (abac_minres_solve), including members that join a
group while others are already iterating, and an FP64 member must match the oracle.
Every case prints its identity before touching the GPU.
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
TOL = 1e-8
MAXIT = 200

# (nx, ny, nt, alpha, batch): 1D and 2D, square grids on the fused x-y passes and
# non-square ones on the separate passes, several batches, x lengths 128 .. 4096
FP32_MIX = [(255, 0, 64, 1e-2, 1), (1023, 0, 64, 1e-3, 2), (63, 63, 64, 1e-3, 1), (31, 15, 32, 1e-3, 1),
            (2047, 0, 16, 1e-3, 1), (127, 127, 128, 1e-2, 1)]
FP64_MIX = [(255, 0, 64, 1e-3, 1), (63, 63, 64, 1e-2, 1), (127, 63, 32, 1e-3, 2), (1023, 0, 16, 1e-3, 1)]


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _inputs(nx, ny, nt, batch, seed):
    srcs = [synth.random_source(nx, ny, nt, seed=seed + b) for b in range(batch)]
    src = np.stack([s[0] for s in srcs])
    z = np.stack([s[1] for s in srcs])
    return (torch.from_numpy(src).to(DEV), torch.from_numpy(z).to(DEV), torch.from_numpy(z.copy()).to(DEV))


def _plan(case, prec):
    from paper_2306_03574_amd import Plan
    nx, ny, nt, alpha, batch = case
    return Plan(nx, ny, nt, alpha=alpha, prec=prec, batch=batch, device=DEV)


def _solo(case, prec, seed):
    _say(f"solo {case} {prec}")
    p = _plan(case, prec)
    f = p.build_rhs(*_inputs(case[0], case[1], case[2], case[4], seed))
    u, iters, relres, status = p.solve(f, tol=TOL, maxit=MAXIT)
    return _host(f), _host(u), iters, relres, status


def _step(g, k, persistent, blocks=0):
    if persistent:
        g.run(k, blocks=blocks)
    else:
        g.advance(k)


def _run_group(g, plans, limit, persistent=False, chunk=1, blocks=0):
    for _ in range(0, limit, chunk):
        _step(g, chunk, persistent, blocks)
        torch.cuda.synchronize()
        if all(p.poll() for p in plans):
            return
    raise AssertionError("group did not finish")


def _check_members(cases, prec, seeds, late=(), persistent=False, chunk=1, blocks=0):
    """Solve `cases` as one group (those in `late` join after two iterations of the
    others) and compare every member with its solo solve.  persistent: every
    `chunk` iterations run as one persistent launch (abac_group_run) of `blocks`
    workgroups (0: the library's default)."""
    from paper_2306_03574_amd import Group
    solo = [_solo(c, prec, s) for c, s in zip(cases, seeds)]
    plans, fs, us = [], [], []
    for c, s in zip(cases, seeds):
        _say(f"member {c} {prec}")
        p = _plan(c, prec)
        plans.append(p)
        fs.append(p.build_rhs(*_inputs(c[0], c[1], c[2], c[4], s)))
        us.append(p.empty())
    g = Group(device=DEV)
    early = [i for i in range(len(cases)) if i not in late]
    for i in early:
        plans[i].begin(fs[i], us[i], tol=TOL, maxit=MAXIT)
    _say(f"group of {len(early)} {prec} persistent={persistent} chunk={chunk} blocks={blocks}")
    g.set([plans[i] for i in early])
    _step(g, 2, persistent, blocks)
    if late:
        for i in late:
            plans[i].begin(fs[i], us[i], tol=TOL, maxit=MAXIT)
        _say(f"group of {len(cases)} {prec} (late members joined)")
        g.set(plans)
    _run_group(g, plans, MAXIT + 2, persistent, chunk, blocks)
    if persistent:
        assert not g.check()
    for i, (c, p) in enumerate(zip(cases, plans)):
        iters, relres, status = p.finish()
        f0, u0, it0, rr0, st0 = solo[i]
        assert np.array_equal(_host(fs[i]), f0)
        assert status == st0 == [0] * c[4], (c, status, st0)
        assert iters == it0, (c, iters, it0)
        assert relres == rr0, (c, relres, rr0)
        assert np.array_equal(_host(us[i]), u0), (c, float(np.max(np.abs(_host(us[i]) - u0))))
    g.close()
    return solo


def test_group_fp32_mixed_grids_equal_solo():
    _check_members(FP32_MIX, "fp32", [700 + i for i in range(len(FP32_MIX))])


def test_group_fp64_mixed_grids_equal_solo_and_oracle():
    solo = _check_members(FP64_MIX, "fp64", [800 + i for i in range(len(FP64_MIX))])
    # the member on the separate x / y passes against the oracle
    nx, ny, nt, alpha, batch = FP64_MIX[2]
    g = Grid(nx, ny, nt)
    f0, u0, it0, _, _ = solo[2]
    L = L_matrix(g)
    for b in range(batch):
        _say(f"oracle solve {FP64_MIX[2]} rhs {b}")
        ref = mr.minres(lambda v: aao.apply_A(g, v, L), lambda y: pc.apply_Pinv(g, alpha, y),
                        aao.reverse_time(f0[b]), tol=TOL, maxit=MAXIT)
        assert ref.converged and it0[b] == ref.iters
        assert np.max(np.abs(u0[b] - ref.x)) / np.max(np.abs(ref.x)) < 1e-10


def test_group_members_joining_late_equal_solo():
    """Continuous batching: two members start, two more join after two iterations."""
    cases = [FP32_MIX[0], FP32_MIX[2], FP32_MIX[3], FP32_MIX[1]]
    _check_members(cases, "fp32", [900, 901, 902, 903], late=(2, 3))


def test_group_rejects_what_it_cannot_run():
    from paper_2306_03574_amd import Group
    from paper_2306_03574_amd.abac import AbacError, EINVAL
    _say("group rejections")
    g = Group(device=DEV)
    small = _plan((63, 0, 64, 1e-3, 1), "fp64")     # the one-launch small-problem path
    assert small.tiles()["small"] > 0
    f = small.build_rhs(*_inputs(63, 0, 64, 1, 5))
    u = small.empty()
    small.begin(f, u, tol=TOL, maxit=MAXIT)
    with pytest.raises(AbacError) as e:
        g.set([small])
    assert e.value.status == EINVAL
    small.finish()
    idle = _plan((255, 0, 64, 1e-3, 1), "fp64")     # no solve begun
    with pytest.raises(AbacError):
        g.set([idle])
    a = _plan((255, 0, 64, 1e-3, 1), "fp64")
    b = _plan((255, 0, 64, 1e-3, 1), "fp32")        # another transform precision
    for p in (a, b):
        p.begin(p.build_rhs(*_inputs(255, 0, 64, 1, 6)), p.empty(), tol=TOL, maxit=MAXIT)
    with pytest.raises(AbacError):
        g.set([a, b])
    with pytest.raises(AbacError):
        g.set([a, a])
    a.finish()
    b.finish()
    g.close()


def test_persistent_group_fp32_mixed_grids_equal_solo():
    """One persistent launch per iteration (abac_group_run): bitwise the solo solves."""
    _check_members(FP32_MIX, "fp32", [700 + i for i in range(len(FP32_MIX))], persistent=True)


def test_persistent_group_fp64_mixed_grids_equal_solo():
    _check_members(FP64_MIX, "fp64", [800 + i for i in range(len(FP64_MIX))], persistent=True)


def test_persistent_group_many_iterations_per_launch_with_late_members():
    """Eight iterations per launch; two members join after two iterations of the others;
    members that stop skip their work in the launches that follow."""
    cases = [FP32_MIX[0], FP32_MIX[2], FP32_MIX[3], FP32_MIX[1]]
    _check_members(cases, "fp32", [900, 901, 902, 903], late=(2, 3), persistent=True, chunk=8)


def test_persistent_group_1d_only_mix_equal_solo():
    """1D members only: the y steps have no blocks and their barriers are skipped."""
    cases = [(255, 0, 64, 1e-3, 1), (1023, 0, 64, 1e-2, 2), (2047, 0, 16, 1e-3, 1)]
    _check_members(cases, "fp64", [930, 931, 932], persistent=True, chunk=3)


@pytest.mark.parametrize("blocks", [1, 8, 40, 1024])
def test_persistent_group_any_grid_size_equals_solo(blocks):
    """Grids from one workgroup (every logical block in turn, no waiting at barriers) to
    more than the largest step's blocks (capped): the same results."""
    _check_members([FP64_MIX[1], FP64_MIX[2]], "fp64", [920, 921], persistent=True, chunk=4, blocks=blocks)


def test_persistent_group_timeout_is_reported_and_recovered():
    """A barrier wait limit of zero (forced from the host) makes the waiting blocks give
    up at the first barrier: the launch ends, abac_group_check reports it, and the next
    launch of the same group, with fresh members, again matches the solo solves."""
    from paper_2306_03574_amd import Group
    case = FP32_MIX[2]
    g = Group(device=DEV)
    p = _plan(case, "fp32")
    _say(f"persistent timeout {case}")
    p.begin(p.build_rhs(*_inputs(case[0], case[1], case[2], case[4], 11)), p.empty(), tol=TOL, maxit=MAXIT)
    g.set([p])
    g.run(1, timeout_s=1e-12)
    torch.cuda.synchronize()
    assert g.check()
    assert not g.check()        # the flag was cleared
    from paper_2306_03574_amd.abac import AbacError
    try:
        p.finish()              # the member's state is invalid; only its release is checked
    except AbacError:
        pass
    g.close()
    _check_members([FP32_MIX[0], FP32_MIX[3]], "fp32", [910, 911], persistent=True)


def test_persistent_group_random_mixes_equal_list_launches():
    """Twelve seeded random mixes (1 to 4 members, FP32 or FP64), grid sizes and iteration
    counts: the persistent launch gives bitwise the iterates of one launch per step."""
    import random
    from paper_2306_03574_amd import Group
    pool = [(255, 0, 64, 1e-3, 1), (1023, 0, 64, 1e-2, 2), (63, 63, 64, 1e-3, 1), (31, 15, 32, 1e-3, 1),
            (127, 63, 32, 1e-3, 2), (2047, 0, 16, 1e-3, 1), (127, 127, 128, 1e-2, 1), (63, 63, 256, 1e-2, 1)]
    rng = random.Random(2024)
    for trial in range(12):
        prec = rng.choice(["fp32", "fp64"])
        cases = rng.sample(pool, rng.randint(1, 4))
        blocks = rng.choice([0, 1, 8, 40, 128, 1024])
        iters = rng.randint(1, 5)
        _say(f"random trial {trial}: {prec} blocks {blocks} iterations {iters} {cases}")
        out = {}
        for mode in ("advance", "run"):
            plans, us = [], []
            for i, c in enumerate(cases):
                p = _plan(c, prec)
                p.begin(p.build_rhs(*_inputs(c[0], c[1], c[2], c[4], 1000 + 10 * trial + i)), u := p.empty(),
                        tol=1e-30, maxit=1000)
                plans.append(p)
                us.append(u)
            g = Group(device=DEV)
            g.set(plans)
            if mode == "advance":
                g.advance(iters)
            else:
                g.run(iters, blocks=blocks)
                assert not g.check()
            out[mode] = [(p.finish(), _host(u)) for p, u in zip(plans, us)]
            g.close()
        for (ra, ua), (rb, ub) in zip(out["advance"], out["run"]):
            assert ra == rb, (trial, ra, rb)
            assert np.array_equal(ua, ub), (trial, float(np.max(np.abs(ua - ub))))
