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
The transforms' own rounding, not the weights, sets the count.

    python tests/fp32_rounding_study.py 1e-2 passes

mirrors the GPU's passes instead, z = Sx Sy [K Y K Y] Sy Sx r with the scratch rounded
to single precision between passes, and sets each pass's arithmetic (x DSTs, y DSTs,
time FFTs) to single or double precision.  Measured at alpha = 1e-2 (the same counts in
two runs): all double 8, all single 11, time pass double 8, x and y double 9, x double 9.
An earlier draft of this emulation, differing only in where arrays were copied, gave
9, 10 and 11 for the rows with a single-precision time pass: with single-precision
time-pass arithmetic the count moves between 9 and 11 with the rounding details, and
only double-precision time-pass arithmetic (8 in every variant) brings it within 2 of 6."""
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

def make_pass_pinv(x32, y32, t32):
    """The GPU's pass structure with single-precision scratch between passes; each
    pass's arithmetic in single (True) or double precision."""
    M64 = pc.principal_inv_sqrt(pc.mu_table(g, alpha))
    d64 = pc.time_scaling(nt, alpha)
    M = M64.astype(np.complex64) if t32 else M64
    ct = np.complex64 if t32 else np.complex128
    rt = np.float32 if t32 else np.float64
    d = d64.astype(rt)

    def dst(v, axis, p32):
        return sfft.dst(np.asarray(v, dtype=np.float32 if p32 else np.float64), type=1, axis=axis, norm="ortho",
                        workers=-1)

    def K(v):
        v = (v * d[:, None, None]).astype(ct)
        v = sfft.ifft((M * sfft.fft(v, axis=0, workers=-1)).astype(ct), axis=0, workers=-1)
        return (v.real.astype(rt) / d[:, None, None]).astype(rt)

    def pinv(r):
        v = dst(r, 2, x32).astype(np.float32)
        v = dst(v, 1, y32).astype(np.float32)
        w = K(K(v.astype(rt)[::-1])[::-1]).astype(np.float32)
        w = dst(w, 1, y32).astype(np.float32)
        return np.asarray(dst(w, 2, x32), dtype=np.float64)
    return pinv


def main_passes():
    src, p0, p1, _ = synth.manufactured_2d(nx, ny, nt)
    f = aao.build_rhs(g, src, p0, p1)
    L = L_matrix(g)
    for name, x32, y32, t32 in [("all double", False, False, False), ("all single", True, True, True),
                                ("time double", True, True, False), ("x, y double", False, False, True),
                                ("x double", False, True, True)]:
        P = make_pass_pinv(x32, y32, t32)
        t0 = time.time()
        r = mr.minres(lambda v: aao.apply_A(g, v, L), P, aao.reverse_time(f), tol=1e-8, maxit=60)
        print(f"alpha {alpha}: passes, {name:14s} iters {r.iters} converged {r.converged} ({time.time() - t0:.0f} s)",
              flush=True)


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
    main_passes() if len(sys.argv) > 2 and sys.argv[2] == "passes" else main()
