"""Writes dims_iterations.txt: the oracle's iteration counts for the
dimension study of Sec. 4.2 at d = 6, P = 1024 (levels (3,3,3,3,3,3),
117,649 unknowns): isotropic levels floor((S + log2 P) / d), S = 8,
q = 2^(S-4) = 16, gamma = 1/2, omega-weighted balanced preconditioner, the
Sec. 4 protocol (b = 0, random start with ||x0||_A = 1 from splitmix64 seed
11, stop when the energy norm of the error falls below 1e-8); PCG, and
Richardson with the damping 2 / (lmin + lmax) from the oracle's 150-step
Lanczos estimate (seed 99).  Both curves.  Calls the oracle only.

Usage: python tests/golden/make_dims_iterations.py   (about 10 minutes on 8 cores)
"""
import os
import sys
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from seeded_inputs import uniform_pm1  # noqa: E402
from oracle.grid import Grid  # noqa: E402
from oracle.schwarz import OracleSchwarz  # noqa: E402
from oracle import solvers  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dims_iterations.txt")
CASES = [(6, 1024)]


def main():
    rows = []
    for d, P in CASES:
        lv = (int((8 + int(np.log2(P))) // d),) * d
        g = Grid(levels=lv)
        for curve in ("zorder", "hilbert"):
            O = OracleSchwarz(g, P, Fraction(1, 2), q=16, curve=curve)
            x0 = solvers.paper_start(O.A_nat, 11, g.N)
            zero = np.zeros(g.N)
            it_p = solvers.pcg(O.A_nat, zero, O.apply, x0=x0, energy_tol=1e-8)[1]
            a, b = solvers.cg_coefficients(O.A_nat, uniform_pm1(99, g.N), O.apply, 150)
            xi, _ = solvers.optimal_damping(*solvers.lanczos_extremes(a, b))
            it_r = solvers.richardson(O.A_nat, zero, O.apply, xi, x0=x0, energy_tol=1e-8)[1]
            rows.append((d, P, curve, it_p, it_r, xi))
            print(d, P, curve, it_p, it_r, xi, flush=True)
    with open(OUT, "w") as fh:
        fh.write("# Oracle iteration counts of the Sec. 4.2 dimension study (isotropic levels\n"
                 "# floor((8 + log2 P) / d), q = 16, gamma = 1/2, omega-weighted balanced, b = 0,\n"
                 "# start seed 11 scaled to ||x0||_A = 1, energy norm of the error to 1e-8).\n"
                 "# Written by make_dims_iterations.py (oracle only).\n"
                 "# d  P  curve  pcg  richardson  xi\n")
        for r in rows:
            fh.write("%d %d %s %d %d %.17g\n" % r)


if __name__ == "__main__":
    main()
