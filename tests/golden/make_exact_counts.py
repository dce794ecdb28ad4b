"""Writes exact_minres_counts.json: exact-arithmetic MINRES-I iteration counts (tol
1e-6, x_0 = 0) for the unpreconditioned columns of Tables 1 and 3 at the sizes the
tests use.  Calls only the oracle.  Run from the repository root:
``python tests/golden/make_exact_counts.py``."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.discretization import Grid  # noqa: E402
from oracle import allatonce as aao, examples as ex, minres as mr, varcoef as vc  # noqa: E402


def example1(lt, lh):
    g = Grid(2 ** lh - 1, 2 ** lh - 1, 2 ** lt)
    src, p0, p1, _ = ex.example1_data(g)
    b = aao.reverse_time(aao.build_rhs(g, src, p0, p1))
    return mr.exact_minres_count(lambda v: aao.apply_A(g, v.reshape(g.shape)), b, 1e-6, 4000)


def example2(lt, lh):
    g = Grid(2 ** lh - 1, 2 ** lh - 1, 2 ** lt)
    _, axh, ayh = vc.coefficient_samples(g, vc.example2_coefficient)
    La = vc.L_var(g, axh, ayh)
    src, p0, p1, _ = vc.example2_data(g)
    b = aao.reverse_time(vc.build_rhs_var(g, src, p0, p1, La))
    return mr.exact_minres_count(lambda v: aao.reverse_time(vc.apply_T_var(g, v.reshape(g.shape), La)), b, 1e-6, 4000)


def main():
    out = {
        "citation": "exact-arithmetic counts for the MINRES-I columns of Table 1 (Example 1) and "
                    "Table 3 (Example 2), tol 1e-6; written by make_exact_counts.py from the oracle",
        "example1": {f"{lt},{lh}": example1(lt, lh) for lt, lh in [(4, 4), (4, 5)]},
        "example2": {f"{lt},{lh}": example2(lt, lh) for lt, lh in [(4, 4)]},
    }
    with open(os.path.join(HERE, "exact_minres_counts.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
