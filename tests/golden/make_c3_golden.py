"""Writes c3_oracle.json: the FP64 oracle's MINRES solve of the 511^2 x 512 workload
(Gaussian random-field source, seed 3, ell = 0.1, zero initial data; alpha = 1e-3,
tol = 1e-8, x_0 = 0), stored so that GPU tests at this size can compare against the
oracle without repeating its several-minute solve.

Stored: the iteration count, the explicit relative residual, the recurrence residual
history, the iterate's max-norm and 2-norm, and the iterate at a fixed sample of
entries (a seeded random set, the whole time line through the centre point and the
whole x-row through the centre of the middle level).  Also the oracle's P_alpha^{-1}
applied to the right-hand side at the same entries.

Calls only the oracle and the seeded input recipe.  Run from the repository root
(several minutes, about 25 GB of host memory):
``python tests/golden/make_c3_golden.py``."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.discretization import Grid, L_matrix  # noqa: E402
from oracle import allatonce as aao, minres as mr, preconditioner as pc  # noqa: E402

NX, NY, NT, ALPHA, TOL, SEED = 511, 511, 512, 1e-3, 1e-8, 3
SAMPLE_SEED, NSAMPLE = 20240, 4096


def sample_indices(shape):
    """Flat indices of the stored entries: NSAMPLE seeded random ones, the time line
    through the centre point, the x-row through the centre of the middle level."""
    nt, ny, nx = shape
    rng = np.random.default_rng(SAMPLE_SEED)
    rand = rng.choice(nt * ny * nx, size=NSAMPLE, replace=False)
    tline = np.arange(nt) * (ny * nx) + (ny // 2) * nx + nx // 2
    xrow = (nt // 2) * (ny * nx) + (ny // 2) * nx + np.arange(nx)
    return np.unique(np.concatenate([rand, tline, xrow]))


def main():
    t0 = time.perf_counter()
    g = Grid(NX, NY, NT, 1.0)
    src, p0, p1 = synth.gaussian_field_source(NX, NY, NT, seed=SEED)
    f = aao.build_rhs(g, src, p0, p1)
    del src
    L = L_matrix(g)
    b = aao.reverse_time(f)
    idx = sample_indices(g.shape)
    pb = pc.apply_Pinv(g, ALPHA, b).reshape(-1)[idx]
    calls = [0]

    def A(v):
        calls[0] += 1
        print(f"A call {calls[0]}  {time.perf_counter() - t0:.0f} s", flush=True)
        return aao.apply_A(g, v, L)

    res = mr.minres(A, lambda y: pc.apply_Pinv(g, ALPHA, y), b, tol=TOL, maxit=200)
    x = res.x.reshape(-1)
    host_res = float(np.linalg.norm(f - aao.apply_T(g, res.x, L)) / np.linalg.norm(f))
    out = {
        "citation": "FP64 oracle solve of the 511^2 x 512 workload (Section 3 solver set-up: MINRES with "
                    "the ABAC preconditioner, zero initial guess, true-residual stop); written by "
                    "make_c3_golden.py from the oracle",
        "grid": [NX, NY, NT], "alpha": ALPHA, "tol": TOL, "source": "gaussian_field", "seed": SEED,
        "iters": int(res.iters), "converged": bool(res.converged), "relres_explicit": float(res.relres),
        "relres_T": host_res,
        "relres_history": [float(v) for v in res.relres_history],
        "x_maxabs": float(np.max(np.abs(x))), "x_norm2": float(np.linalg.norm(x)),
        "b_norm2": float(np.linalg.norm(b)), "f_maxabs": float(np.max(np.abs(f))),
        "sample_seed": SAMPLE_SEED, "n_random": NSAMPLE,
        "index": [int(i) for i in idx],
        "x": [float(v) for v in x[idx]],
        "pinv_b": [float(v) for v in pb],
        "pinv_b_maxabs_sampled": float(np.max(np.abs(pb))),
        "oracle_seconds": round(time.perf_counter() - t0, 1),
    }
    with open(os.path.join(HERE, "c3_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"iters {res.iters} relres {res.relres:.3e} ({out['oracle_seconds']} s)", flush=True)


if __name__ == "__main__":
    main()
