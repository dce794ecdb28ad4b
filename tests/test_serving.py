"""Request server and seeded device sources.

CPU tests: the numpy Philox N(0,1) stream is statistically sound and seed-separated;
the server rejects requests larger than its budget without a GPU.
GPU tests: the device generator equals the numpy one; served solves match the oracle;
every result is the same alone and in a mix of concurrent requests; admission never
exceeds the byte budget.
"""
import ctypes

import numpy as np
import pytest

import synth
from synth.philox import normal_stream


def test_philox_normal_stream_statistics():
    x = normal_stream(1_000_003, seed=5001)
    assert abs(x.mean()) < 5e-3 and abs(x.var() - 1) < 5e-3
    assert abs(np.mean(x ** 3)) < 1e-2 and abs(np.mean(x ** 4) - 3) < 3e-2
    # first n values do not depend on the stream length; seeds give different streams
    assert np.array_equal(normal_stream(10, 5001), x[:10])
    y = normal_stream(1000, 5002)
    assert abs(np.corrcoef(x[:1000], y)[0, 1]) < 0.1


def test_server_rejects_request_over_budget_without_gpu():
    from paper_2306_03574_amd.abac import load_library
    lib = load_library()
    h = ctypes.c_void_p()
    assert lib.abac_server_create(1 << 20, 4, ctypes.byref(h)) == 0
    t = ctypes.c_longlong(0)
    st = lib.abac_server_submit(h, 255, 255, 256, 1.0, 1e-3, 1, 7, 1e-8, 100, 0.0, 0, ctypes.byref(t))
    assert st == -6            # ABAC_EBUDGET
    st = lib.abac_server_submit(h, 254, 0, 64, 1.0, 1e-3, 1, 7, 1e-8, 100, 0.0, 0, ctypes.byref(t))
    assert st == -1            # ABAC_EINVAL (nx+1 not a power of two)
    assert lib.abac_server_destroy(h) == 0


@pytest.mark.gpu
def test_device_normals_match_numpy_philox():
    import torch
    from paper_2306_03574_amd.abac import fill_normal
    print("[case] fill_normal n=100003 seed=5007", flush=True)
    out = torch.empty(100003, dtype=torch.float64, device="cuda:0")
    fill_normal(out, 5007)
    torch.cuda.synchronize()
    ref = normal_stream(100003, 5007)
    assert np.max(np.abs(out.cpu().numpy() - ref)) < 1e-12


def _oracle_solve(nx, ny, nt, alpha, seed, tol=1e-8):
    from oracle.discretization import Grid, L_matrix
    from oracle import allatonce as aao, preconditioner as pc, minres as mr
    g = Grid(nx, ny, nt)
    src = normal_stream(g.N, seed).reshape(g.shape)
    z = np.zeros(g.level_shape)
    f = aao.build_rhs(g, src, z, z)
    L = L_matrix(g)
    return mr.minres(lambda v: aao.apply_A(g, v, L), lambda y: pc.apply_Pinv(g, alpha, y), aao.reverse_time(f),
                     tol=tol, maxit=300)


@pytest.mark.gpu
@pytest.mark.parametrize("nx,ny,nt,alpha,prec", [(255, 0, 64, 1e-2, "fp64"), (63, 63, 64, 1e-3, "fp64"),
                                                 (255, 0, 64, 1e-3, "fp32")])
def test_served_solve_matches_oracle(nx, ny, nt, alpha, prec):
    from paper_2306_03574_amd.serve import Server
    print(f"[case] served nx={nx} ny={ny} nt={nt} alpha={alpha} prec={prec}", flush=True)
    srv = Server(8 << 30, 4)
    n = nt * nx * max(ny, 1)
    t = srv.submit(nx, ny, nt, alpha, seed=5003, prec=prec, keep=True)
    res = srv.drain([t], n_unknowns=n, timeout=120)[t]
    ref = _oracle_solve(nx, ny, nt, alpha, 5003)
    assert res["status"] == 0 and res["relres"] <= 1e-8
    err = np.max(np.abs(res["u"] - ref.x.reshape(-1))) / np.max(np.abs(ref.x))
    if prec == "fp64":
        assert res["iters"] == ref.iters and err < 1e-10
    else:
        assert res["iters"] <= ref.iters + 2 and err < 1e-6
    srv.close()


MIX = [(255, 0, 64, 1e-2), (1023, 0, 256, 1e-3), (63, 63, 64, 1e-2), (127, 127, 64, 1e-3), (4095, 0, 64, 1e-3),
       (255, 0, 1024, 1e-2), (63, 63, 256, 1e-3), (127, 127, 256, 1e-2)]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_same_result_alone_and_in_the_mix(prec):
    """Each request's solution is bitwise the same whether it runs alone or admitted
    while seven other requests of different shapes are on the GPU."""
    from paper_2306_03574_amd.serve import Server
    print(f"[case] alone-vs-mix prec={prec}", flush=True)
    sizes = {i: nt * nx * max(ny, 1) for i, (nx, ny, nt, a) in enumerate(MIX)}
    alone = {}
    srv = Server(64 << 30, 1)
    for i, (nx, ny, nt, a) in enumerate(MIX):
        if prec == "fp64" and nx == 4095:
            continue
        t = srv.submit(nx, ny, nt, a, seed=5100 + i, prec=prec, keep=True)
        alone[i] = srv.drain([t], n_unknowns=sizes[i], timeout=120)[t]
    srv.close()
    srv = Server(64 << 30, 8)
    tickets = {}
    for i, (nx, ny, nt, a) in enumerate(MIX):
        if i in alone:
            tickets[srv.submit(nx, ny, nt, a, seed=5100 + i, prec=prec, keep=True)] = i
            srv.step()                 # later requests arrive while earlier ones run
    mixed = srv.drain(list(tickets), n_unknowns={t: sizes[i] for t, i in tickets.items()}, timeout=300)
    srv.close()
    for t, i in tickets.items():
        a, m = alone[i], mixed[t]
        assert a["status"] == m["status"] == 0 and a["relres"] <= 1e-8
        assert a["iters"] == m["iters"]
        assert np.array_equal(a["u"], m["u"]), MIX[i]


@pytest.mark.gpu
def test_admission_respects_budget_and_queues():
    """With a budget that holds two large slots at most, a burst of requests queues,
    all complete, and the server never holds more than its budget."""
    from paper_2306_03574_amd.serve import Server
    from paper_2306_03574_amd.abac import workspace_bytes
    print("[case] admission budget", flush=True)
    nx, ny, nt = 127, 127, 256
    n = nt * nx * ny
    slot = workspace_bytes(nx, ny, nt, "fp32") + 2 * 8 * n + 8 * nx * ny + 4096
    budget = int(2.5 * slot)
    srv = Server(budget, 8)
    tickets = [srv.submit(nx, ny, nt, 1e-3, seed=5200 + i, prec="fp32") for i in range(6)]
    peak_active = 0
    out = {}
    while len(out) < len(tickets):
        a, q = srv.step()
        peak_active = max(peak_active, a)
        assert srv.bytes_in_use() <= budget
        for t in tickets:
            if t not in out:
                r = srv.result(t)
                if r is not None:
                    out[t] = r
    assert peak_active <= 2
    assert all(r["status"] == 0 and r["relres"] <= 1e-8 for r in out.values())
    srv.close()


@pytest.mark.gpu
def test_group_lane_gives_the_same_results():
    """The server's group lane (requests of up to 300000 unknowns advance together, one
    launch per MINRES step) returns bitwise the solutions, counts and residuals of the
    server without it, for a mix of shapes submitted together and while others run."""
    from paper_2306_03574_amd.serve import Server
    mix = [(255, 0, 64, 1e-2), (1023, 0, 256, 1e-3), (63, 63, 64, 1e-2), (255, 0, 1024, 1e-3), (4095, 0, 64, 1e-3),
           (63, 63, 256, 1e-3), (127, 127, 64, 1e-3), (1023, 0, 64, 1e-2)]
    out = {}
    for lane in (0, 300_000):
        print(f"[case] server group lane {lane}", flush=True)
        srv = Server(64 << 30, 16, lane)
        first = [srv.submit(nx, ny, nt, a, seed=5100 + i, keep=True) for i, (nx, ny, nt, a) in enumerate(mix[:4])]
        for _ in range(3):
            srv.step()
        later = [srv.submit(nx, ny, nt, a, seed=5104 + i, keep=True) for i, (nx, ny, nt, a) in enumerate(mix[4:])]
        tickets = first + later
        sizes = {t: nt * nx * max(ny, 1) for t, (nx, ny, nt, a) in zip(tickets, mix)}
        res = srv.drain(tickets, n_unknowns=sizes, timeout=120)
        out[lane] = [res[t] for t in tickets]
        srv.close()
    for a, b, shape in zip(out[0], out[300_000], mix):
        assert a["status"] == b["status"] == 0 and a["relres"] <= 1e-8, shape
        assert a["iters"] == b["iters"] and a["relres"] == b["relres"], shape
        assert np.array_equal(a["u"], b["u"]), shape
    # one lane member against the oracle (FP32 transforms: count within 2)
    ref = _oracle_solve(255, 0, 64, 1e-2, 5100)
    assert abs(out[300_000][0]["iters"] - ref.iters) <= 2
