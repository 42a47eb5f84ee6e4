"""Write the stored expected correlators of tests/golden/ with the FP64 oracle.

Calls only oracle/ (and synth/ for the seeded inputs).  Each file holds
C_PP(t) = -sum_x tr[S^+ S] (the correlator of the heavy-quark section) of the
12-column point-source propagator at the origin, restored from the solution
of the preconditioned system (eq. linsysprec) solved by the oracle's
BiCGStab to a relative residual of 1e-13 with the paper's periodic-time
profile (eq. pbcalpha) at alpha0 = 0.4, which keeps every timeslice resolved.

Usage: python tests/golden/make_golden.py [--threads N]
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def golden_16c32(threads):
    cfg = synth.config("su3_16c32")
    dims, M = cfg["dims"], cfg["masses"][0]
    oracle.set_threads(threads)
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    alpha = synth.alpha_table("cosh", dims[0], 0.4)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    cpp = np.zeros(dims[0])
    iters = []
    for c in range(12):
        t0 = time.time()
        S, info = oracle.solve(U, C, M, eta[c], alpha=alpha, r=1e-13)
        cpp += oracle.cpp(S)
        iters.append(info["iters"])
        print(f"column {c}: {info['iters']} iterations, relres {info['relres_prec']:.2e}, {time.time() - t0:.1f} s",
              flush=True)
    path = os.path.join(HERE, "cpp_su3_16c32_M0.5.txt")
    with open(path, "w") as f:
        f.write("# C_PP(t), t = 0..31: 16^3x32 synthetic SU(3) field (eps 0.3, seed 1632), c_sw 1.6, M 0.5,\n")
        f.write("# antiperiodic time, 12 point-source columns at the origin.  FP64 oracle BiCGStab to 1e-13 on the\n")
        f.write("# preconditioned system (cosh profile, alpha0 0.4), restored.  Written by tests/golden/make_golden.py\n")
        f.write(f"# oracle iterations per column: {iters}\n")
        for t, v in enumerate(cpp):
            f.write(f"{t} {v:.17e}\n")
    print("wrote", path)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    golden_16c32(ap.parse_args().threads)
