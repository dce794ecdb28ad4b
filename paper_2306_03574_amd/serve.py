"""Python front end of the native request server (``abac_server_*`` in libabac.so).

The scheduling (admission by HBM budget, continuous batching at iteration
granularity, per-request streams, slot caching) runs in the library; this module
only submits requests at their arrival times and collects results.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from .abac import load_library, _check, PREC, OK, EAGAIN, AbacError


class Server:
    def __init__(self, budget_bytes: int, max_active: int = 16, group_max_unknowns: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        _check(self._lib.abac_server_create(int(budget_bytes), int(max_active), ctypes.byref(h)), "abac_server_create")
        self._h = h
        if group_max_unknowns:
            _check(self._lib.abac_server_group_lane(self._h, int(group_max_unknowns)), "abac_server_group_lane")

    def clock(self) -> float:
        return float(self._lib.abac_server_clock(self._h))

    def submit(self, nx, ny, nt, alpha, seed, prec="fp32", tol=1e-8, maxit=500, T=1.0, arrival=None, keep=False):
        t = ctypes.c_longlong(0)
        arrival = self.clock() if arrival is None else arrival
        _check(self._lib.abac_server_submit(self._h, nx, ny, nt, float(T), float(alpha), PREC[prec], int(seed),
                                            float(tol), int(maxit), float(arrival), 1 if keep else 0,
                                            ctypes.byref(t)), "abac_server_submit")
        return t.value

    def step(self):
        a, q = ctypes.c_int(0), ctypes.c_int(0)
        _check(self._lib.abac_server_step(self._h, ctypes.byref(a), ctypes.byref(q)), "abac_server_step")
        return a.value, q.value

    def result(self, ticket, n_unknowns=None):
        """None while pending; else dict(iters, relres, status, latency[, u])."""
        it, st = ctypes.c_int(0), ctypes.c_int(0)
        rr, lat = ctypes.c_double(0), ctypes.c_double(0)
        u = np.empty(n_unknowns) if n_unknowns else None
        ptr = ctypes.c_void_p(u.ctypes.data) if u is not None else None
        s = self._lib.abac_server_result(self._h, int(ticket), ptr, ctypes.byref(it), ctypes.byref(rr),
                                         ctypes.byref(st), ctypes.byref(lat))
        if s == EAGAIN:
            return None
        _check(s, "abac_server_result")
        out = {"iters": it.value, "relres": rr.value, "status": st.value, "latency": lat.value}
        if u is not None:
            out["u"] = u
        return out

    def bytes_in_use(self) -> int:
        return int(self._lib.abac_server_bytes_in_use(self._h))

    def drain(self, tickets, n_unknowns=None, timeout=600.0):
        """Step until every ticket has a result; returns {ticket: result}."""
        out = {}
        pending = list(tickets)
        t_end = time.perf_counter() + timeout
        while pending:
            self.step()
            rest = []
            for t in pending:
                r = self.result(t, n_unknowns.get(t) if isinstance(n_unknowns, dict) else n_unknowns)
                if r is None:
                    rest.append(t)
                else:
                    out[t] = r
            pending = rest
            if time.perf_counter() > t_end:
                raise TimeoutError(f"{len(pending)} requests still pending")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.abac_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_trace(trace, budget_bytes, max_active=16, prec="fp32", tol=1e-8, maxit=500, progress=None,
              warm_classes=(), group_max_unknowns=0):
    """Replay a Poisson trace (list of dicts with arrival, nx, ny, nt, alpha, seed):
    each request is submitted when the server clock reaches its arrival time.
    group_max_unknowns > 0 runs requests up to that size in the server's group lane.
    Returns (per-request results in trace order, wall seconds from the first arrival
    to the last completion)."""
    srv = Server(budget_bytes, max_active, group_max_unknowns)
    if warm_classes:
        # one untimed solve per shape class: the server keeps their plans and graphs cached
        warm = [srv.submit(nx, ny, nt, a, seed=1, prec=prec, tol=tol, maxit=maxit) for (nx, ny, nt, a) in warm_classes]
        srv.drain(warm, timeout=600)
    t0 = srv.clock()
    tickets = [None] * len(trace)
    results = [None] * len(trace)
    nxt = 0
    done = 0
    last_report = time.perf_counter()
    while done < len(trace):
        now = srv.clock() - t0
        while nxt < len(trace) and trace[nxt]["arrival"] <= now:
            r = trace[nxt]
            tickets[nxt] = srv.submit(r["nx"], r["ny"], r["nt"], r["alpha"], r["seed"], prec=prec, tol=tol,
                                      maxit=maxit, arrival=t0 + r["arrival"])
            nxt += 1
        srv.step()
        for i in range(len(trace)):
            if tickets[i] is not None and results[i] is None:
                res = srv.result(tickets[i])
                if res is not None:
                    results[i] = res
                    done += 1
        if progress and time.perf_counter() - last_report > 20:
            progress(f"served {done}/{len(trace)}")
            last_report = time.perf_counter()
    wall = srv.clock() - t0
    srv.close()
    return results, wall
