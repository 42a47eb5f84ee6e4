"""Write the stored expected correlators of tests/golden/ with the FP64 oracle.

Calls only oracle/ (and synth/ for the seeded inputs).  Each file holds
C_PP(t) = -sum_x tr[S^+ S] (the correlator of the heavy-quark section) of
point-source propagators at the origin, restored from the solution of the
preconditioned system (eq. linsysprec) solved by the oracle's BiCGStab to a
relative residual of 1e-13.  The correlator does not depend on the profile
(the redefinition of eq. redeft is exact); the profile only keeps every
timeslice resolved in the oracle's own solve.

* 16^3x32 (M 0.5): the 12-column sum, cosh profile alpha0 0.4 (eq. pbcalpha);
* 24^3x48 (M 0.5): the 12-column sum and each column, cosh profile alpha0 0.4;
* 32^3x64 (M 0.01): columns 0 and 7, symmetric exponential profile alpha0 0.1.

Usage: python tests/golden/make_golden.py [--threads N] [--which 16c32,24c48,32c64]
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


def _columns(name, profile, alpha0, cols):
    cfg = synth.config(name)
    dims, M = cfg["dims"], cfg["masses"][0]
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    alpha = synth.alpha_table(profile, dims[0], alpha0)
    per, iters = [], []
    for c in cols:
        t0 = time.time()
        eta = synth.point_source(dims, (0, 0, 0, 0), c // 3, c % 3)
        S, info = oracle.solve(U, C, M, eta, alpha=alpha, r=1e-13)
        per.append(oracle.cpp(S))
        iters.append(info["iters"])
        print(f"{name} column {c}: {info['iters']} iterations, relres {info['relres_prec']:.2e}, "
              f"{time.time() - t0:.1f} s", flush=True)
        del S
    return cfg, np.array(per), iters


def golden_16c32():
    cfg, per, iters = _columns("su3_16c32", "cosh", 0.4, range(12))
    cpp = per.sum(axis=0)
    path = os.path.join(HERE, "cpp_su3_16c32_M0.5.txt")
    with open(path, "w") as f:
        f.write("# C_PP(t), t = 0..31: 16^3x32 synthetic SU(3) field (eps 0.3, seed 1632), c_sw 1.6, M 0.5,\n")
        f.write("# antiperiodic time, 12 point-source columns at the origin.  FP64 oracle BiCGStab to 1e-13 on the\n")
        f.write("# preconditioned system (cosh profile, alpha0 0.4), restored.  Written by tests/golden/make_golden.py\n")
        f.write(f"# oracle iterations per column: {iters}\n")
        for t, v in enumerate(cpp):
            f.write(f"{t} {v:.17e}\n")
    print("wrote", path)


def _write_columns(path, title, cols, per, iters):
    with open(path, "w") as f:
        for line in title:
            f.write("# " + line + "\n")
        f.write(f"# oracle iterations per column: {iters}\n")
        f.write("# columns: t, sum over the listed spin-colour columns, then each column " + " ".join(map(str, cols))
                + "\n")
        for t in range(per.shape[1]):
            f.write(f"{t} {per[:, t].sum():.17e} " + " ".join(f"{v:.17e}" for v in per[:, t]) + "\n")
    print("wrote", path)


def golden_24c48():
    cols = list(range(12))
    cfg, per, iters = _columns("su3_24c48", "cosh", 0.4, cols)
    _write_columns(os.path.join(HERE, "cpp_su3_24c48_M0.5.txt"),
                   ["C_PP(t), t = 0..47: 24^3x48 synthetic SU(3) field (eps 0.25, seed 2448), c_sw 1.6, M 0.5,",
                    "antiperiodic time, point sources at the origin.  FP64 oracle BiCGStab to 1e-13 on the",
                    "preconditioned system (cosh profile, alpha0 0.4), restored.  Written by tests/golden/make_golden.py"],
                   cols, per, iters)


def golden_32c64():
    cols = [0, 7]
    cfg, per, iters = _columns("su3_32c64", "exp_sym", 0.1, cols)
    _write_columns(os.path.join(HERE, "cpp_su3_32c64_M0.01.txt"),
                   ["C_PP(t), t = 0..63: 32^3x64 synthetic SU(3) field (eps 0.2, seed 3264), c_sw 1.6, M 0.01,",
                    "antiperiodic time, point sources at the origin.  FP64 oracle BiCGStab to 1e-13 on the",
                    "preconditioned system (exp(alpha0 min(t, T-t)), alpha0 0.1), restored.",
                    "Written by tests/golden/make_golden.py"],
                   cols, per, iters)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--which", default="16c32,24c48,32c64")
    a = ap.parse_args()
    oracle.set_threads(a.threads)
    for w in a.which.split(","):
        {"16c32": golden_16c32, "24c48": golden_24c48, "32c64": golden_32c64}[w]()
