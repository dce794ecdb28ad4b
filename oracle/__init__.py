"""Plain FP64 CPU oracle for ABAC-preconditioned MINRES on the all-at-once wave system.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything here.
The HIP library never calls it and shares no code, table or constant with it.

Everything is numpy/scipy in float64 and follows the paper (Lin & Hon, "A block
alpha-circulant based preconditioned MINRES method for wave equations"):

* ``discretization`` -- grid, 3/5-point Laplacian, L = I - tau^2/2 Delta_h (Section 1).
* ``allatonce``      -- the block lower-triangular Toeplitz matrix T of eq. (1.2),
                        the right-hand side f of eq. (1.2), the time reversal Y of
                        eqs. (1.3)-(1.4), a time-stepping solve of T u = f.
* ``preconditioner`` -- C_alpha of eqs. (1.5)-(1.6), its eigenvalues (eq. (1.7) and
                        Appendix A), the dense principal square root (eq. (1.8)),
                        P_alpha of eq. (1.9) and the matrix-free apply of P_alpha^{-1}
                        of Section 2.3 (three steps, done twice).
* ``minres``         -- preconditioned MINRES (Section 3 solver set-up) and a
                        brute-force Krylov least-squares minimiser for tiny sizes.
* ``examples``       -- Example 1 of Section 3 and the error E_{tau,h}.

Parity status of each function is stated in its docstring; functions whose
results no paper value, closed form, library routine or invariant pins would say
"parity unpinned" -- none currently do.
"""
