"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a build of orc.c with both sanitizers runs the operator,
the clover term, the solvers (BiCGStab, CGNR, SAP+GCR), the profile
variants, C_PP with a shifted source and the Schroedinger-functional clover
on small lattices with odd extents, in a child process; any report aborts
it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
import oracle, synth
for dims in [(5, 3, 2, 4), (4, 2, 3, 2)]:
    U = synth.gauge_su3(dims, 0.6, 3)
    C = oracle.clover(U, 1.6)
    psi = synth.random_spinor(dims, 4)
    a = synth.alpha_exp(dims[0], 0.4)
    for bc in (-1, 1, 0):
        oracle.apply(U, C, 0.3, psi, alpha=a, bc_t=bc)
        oracle.apply(U, C, 0.3, psi, alpha=a, bc_t=bc, dagger=True)
        oracle.apply_modified(U, C, 0.3, psi, a, bc_t=bc)
    beta = tuple(np.exp(np.linspace(-0.3, 0.3, L)) for L in dims)
    oracle.apply_beta(U, C, 0.3, psi, beta)
    eta = synth.point_sources_12(dims, (1, 0, 0, 0), 2)
    S = np.stack([oracle.solve(U, C, 0.5, eta[c], alpha=a, r=1e-10)[0] for c in range(2)])
    oracle.solve(U, C, 0.5, eta[0], r=1e-10, solver="cgnr")
    oracle.solve(U, C, 0.5, eta[0], beta=beta, r=1e-10)
    oracle.cpp(S, x0_src=1)
U = synth.gauge_su3((4, 4, 4, 4), 0.5, 5)
C = oracle.clover(U, 1.6)
eta = synth.point_sources_12((4, 4, 4, 4), (0, 0, 0, 0), 1)[0]
oracle.solve_sap(U, C, 0.5, eta, (2, 2, 2, 2), r=1e-8)
U_ext = synth.gauge_su3_sf((3, 2, 4, 2), 0.5, 6, (0.1, 0.2, -0.3), (0.2, -0.1, -0.1))
oracle.sf_apply(U_ext, 1.6, 0.4, synth.random_spinor((3, 2, 4, 2), 7), ct_tilde=1.2)
print("sanitized oracle run complete")
"""


def test_oracle_under_asan_and_ubsan(tmp_path):
    from oracle.build import build_sanitized
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's libasan.so not found")
    lib = build_sanitized(str(tmp_path / "liborc_san.so"))
    env = dict(os.environ)
    env.update(ORC_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2",
               PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests")]))
    r = subprocess.run([sys.executable, "-c", SCRIPT], capture_output=True, text=True, env=env, timeout=600,
                       cwd=ROOT)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "sanitized oracle run complete" in r.stdout
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
