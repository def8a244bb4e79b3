"""Writes c2_hilbert_iterations.txt: the oracle's balanced two-level PCG on the
d=3 level (7,6,5) workload (248,031 unknowns, P = 256, gamma = 1/2, Hilbert
curve, omega weights, q by the four-levels-coarser rule), from the balancing
start x0 = F b, to a relative true residual of 1e-9 (Alg. 3 with CG; the
balanced preconditioner of eq. balSW).  Calls the oracle only.

Usage: python tests/golden/make_c2_iterations.py   (about a minute on 8 cores)
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from seeded_inputs import workloads  # noqa: E402
from oracle.grid import Grid  # noqa: E402
from oracle.schwarz import OracleSchwarz  # noqa: E402
from oracle import exact, solvers  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_hilbert_iterations.txt")


def main():
    w = workloads()["c2"]
    g = Grid(levels=w.levels[0])
    f = w.rhs()
    t0 = time.time()
    O = OracleSchwarz(g, w.P, w.gamma, curve="hilbert")
    x0 = O.balancing_start(f)
    x, its, _ = solvers.pcg(O.A_nat, f, O.apply, x0=x0, rtol=w.rtol)
    rel_res = float(np.linalg.norm(f - O.A_nat @ x) / np.linalg.norm(f))
    err = float(np.linalg.norm(x - exact.solve(g, f)) / np.linalg.norm(exact.solve(g, f)))
    with open(OUT, "w") as fh:
        fh.write("# Oracle balanced two-level PCG on the d=3 level (7,6,5) grid, P = 256,\n"
                 "# gamma = 1/2, Hilbert curve, omega weights, q = %d, right-hand side\n"
                 "# splitmix64 seed 2, from the balancing start, to relative residual %.0e.\n"
                 "# Written by make_c2_iterations.py (oracle only).\n"
                 "# iterations  rel_residual  rel_error_vs_exact\n" % (O.q, w.rtol))
        fh.write("%d %.6e %.6e\n" % (its, rel_res, err))
    print(f"{its} iterations, residual {rel_res:.3e}, error {err:.3e}, {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
