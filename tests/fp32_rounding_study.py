"""Which FP32 rounding raises the MINRES count of FP32 transforms on the manufactured
255^2 x 256 problem?  A CPU study, not a test (not collected by pytest; about 2.5
minutes per alpha):

    python tests/fp32_rounding_study.py 1e-2

It applies the fast P^{-1} of Section 2.3 (the oracle's steps) with the transforms
(scipy.fft DST-I and DFT) in single or double precision and the eigenvalue weights
mu^{-1/2} formed in single or double precision, and runs the oracle's MINRES with
each.  Measured: at alpha = 1e-2, 6 iterations in double precision, 10 with single-
precision transforms and double-precision weights, 9 with both single, 8 with
double-precision transforms and single-precision weights; at alpha = 1e-3, 6 and 8, 8, 8.
The transforms' own rounding, not the weights, sets the count."""
import os
import sys
import time

import numpy as np
import scipy.fft as sfft

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle.discretization import Grid, L_matrix, L_eigenvalues  # noqa: E402
from oracle import allatonce as aao, preconditioner as pc, minres as mr  # noqa: E402
import synth  # noqa: E402

nx = ny = 255
nt = 256
alpha = float(sys.argv[1]) if len(sys.argv) > 1 else 1e-2
g = Grid(nx, ny, nt)


def dst2(v):
    """Orthonormal 2D DST-I in the precision of v."""
    return sfft.dstn(v, type=1, axes=(-2, -1), norm="ortho", workers=-1)


def make_pinv(fft32, w32):
    d64 = pc.time_scaling(nt, alpha)
    if w32:
        # mu formed in FP32 from FP32 tables, then 1/sqrt in FP32
        a = np.float32(alpha ** (1.0 / nt))
        k = np.arange(nt)
        w = np.exp(-2j * np.pi * k / nt).astype(np.complex64)
        l1 = (np.float32(1) + a * a * w * w).astype(np.complex64)
        l2 = (np.float32(-2) * a * w).astype(np.complex64)
        lam = L_eigenvalues(g).astype(np.float32)
        mu = lam[None] * l1[:, None, None] + l2[:, None, None]
        M = (np.complex64(1) / np.sqrt(mu.astype(np.complex64))).astype(np.complex64)
    else:
        M = pc.principal_inv_sqrt(pc.mu_table(g, alpha))
        if fft32:
            M = M.astype(np.complex64)
    ct = np.complex64 if fft32 else np.complex128
    rt = np.float32 if fft32 else np.float64
    d = d64.astype(rt)

    def ts(v, s):
        return v * s.reshape((-1, 1, 1))

    def pinv(y):
        # (C^-1/2)^T
        v = dst2(np.asarray(y, dtype=rt))
        v = ts(v, (1 / d).astype(rt)).astype(ct)
        v = sfft.ifft(v, axis=0, workers=-1)
        v = (M * v).astype(ct)
        v = sfft.fft(v, axis=0, workers=-1)
        v = ts(v, d)
        v = (dst2(v.real.astype(rt)) + 1j * dst2(v.imag.astype(rt))).astype(ct)
        # C^-1/2
        v = (dst2(v.real.astype(rt)) + 1j * dst2(v.imag.astype(rt))).astype(ct)
        v = ts(v, d)
        v = sfft.fft(v, axis=0, workers=-1)
        v = (M * v).astype(ct)
        v = sfft.ifft(v, axis=0, workers=-1)
        v = ts(v, (1 / d).astype(rt))
        z = dst2(v.real.astype(rt))
        return z.astype(np.float64)
    return pinv

def main():
    src, p0, p1, _ = synth.manufactured_2d(nx, ny, nt)
    f = aao.build_rhs(g, src, p0, p1)
    L = L_matrix(g)
    for name, fft32, w32 in [("fp64 (oracle-like)", False, False), ("fp32 ffts, fp64 weights", True, False),
                             ("fp32 ffts, fp32 weights", True, True), ("fp64 ffts, fp32 weights", False, True)]:
        P = make_pinv(fft32, w32)
        t0 = time.time()
        r = mr.minres(lambda v: aao.apply_A(g, v, L), P, aao.reverse_time(f), tol=1e-8, maxit=60)
        print(f"alpha {alpha}: {name:28s} iters {r.iters} converged {r.converged} ({time.time() - t0:.0f} s)",
              flush=True)


if __name__ == "__main__":
    main()
