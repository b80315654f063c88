"""Writes the oracle's GRAPE fidelity and gradient for the d = 27 GRAPE
workload (three-transmon chain, six controls, slices of 1 ns) into
tests/golden/grape_d27_M2.txt (M = 2, every slice and control) and
tests/golden/grape_d27_M200_sampled.txt (M = 200, slices 0 and 199, every
control).  Calls only the CPU oracle (block-triangular Frechet derivative,
one 1458 x 1458 Pade build per slice and control) and the seeded input
generator; takes tens of minutes on eight cores.

    python tests/golden/make_grape_d27.py [M2|M200|all]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2603_18052_amd import workloads as W  # noqa: E402


def write(M, slices, name):
    p = W.grape_problem(3, M=M)
    L0 = oracle.liouvillian(p["H0"], p["Lk"])
    Lc = np.stack([oracle.liouvillian(h, p["Lk"][:0]) for h in p["Hc"]])
    t0 = time.time()
    F, g = oracle.grape(L0, Lc, p["u"], p["dt"], p["rho0"].reshape(-1), p["target"].reshape(-1), slices=slices)
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write("# GRAPE fidelity F = Re<w, x_M> and gradient dF/du[m, c] of the d = 27 GRAPE workload\n")
        f.write("# (three-transmon chain, controls x/y per transmon, dt = 1 ns, u seeded as in\n")
        f.write(f"# workloads.grape_problem(3, M={M})), computed by the CPU oracle's block-triangular\n")
        f.write("# Frechet derivative; written by tests/golden/make_grape_d27.py.\n")
        f.write(f"# M {M}\n")
        f.write(f"F {F:.17g}\n")
        f.write("# slice control gradient\n")
        for m in slices:
            for c in range(g.shape[1]):
                f.write(f"{m} {c} {g[m, c]:.17g}\n")
    print(f"{name}: F = {F:.6f}, {len(slices)} slices, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("M2", "all"):
        write(2, [0, 1], "grape_d27_M2.txt")
    if which in ("M200", "all"):
        write(200, [0, 199], "grape_d27_M200_sampled.txt")
