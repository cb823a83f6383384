"""Writes c2_n256_p3_history.txt: the oracle's FP64 stationary V(3,3)
residual history (rho_k = ||b - A x_k|| / ||b||, k = 0..13) for the 2D
viscous-stress benchmark problem at full size (256^2 elements, Q_3,
3,145,728 unknowns, mu = 1 + 0.9 sin 2pi x sin 2pi y, the manufactured
solution of the grid-convergence appendix with Dirichlet data), with the
right-hand side the oracle assembles.  Calls only the oracle and the problem
definition; run from the repository root (about 20 minutes, 30 GB)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth import c2_dirichlet_varmu          # noqa: E402
from oracle import build_hierarchy            # noqa: E402
from oracle.rhs import assemble_rhs           # noqa: E402
from oracle.solvers import Solver             # noqa: E402


def main(cycles=13):
    t0 = time.time()
    prob = c2_dirichlet_varmu(n=256, p=3)
    H = build_hierarchy(prob)
    b = assemble_rhs(prob, H.fine.ops)
    print(f"hierarchy and right-hand side {time.time() - t0:.0f} s", flush=True)
    _, hist = Solver(H).stationary(b, cycles)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_n256_p3_history.txt")
    with open(out, "w") as fh:
        fh.write("# Oracle FP64 stationary V(3,3) residual history, 2D viscous-stress, Dirichlet walls,\n"
                 "# 256^2 elements, Q_3, mu = 1 + 0.9 sin2pi x sin2pi y, manufactured right-hand side\n"
                 "# (written by make_c2_history.py from the oracle alone); k rho_k\n")
        for k, v in enumerate(hist):
            fh.write(f"{k} {v:.17e}\n")
    print(f"wrote {out} after {time.time() - t0:.0f} s: {hist}", flush=True)


if __name__ == "__main__":
    main()
