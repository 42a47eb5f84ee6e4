"""Failure handling of the solvers, with every condition forced from the host
(no kernel is made to fault or hang):

* a BiCGStab breakdown at the first iteration (<rh, M r0> = 0 exactly: the
  caller's clover field cancels 4 + M on the source site of a free field, so
  the Schur operator has a zero diagonal there and the two hops through the
  odd neighbours cancel) is restarted with a pseudo-random shadow residual
  and converges; the oracle recomputes the residual;
* an FP32 / FP16-storage inner solve that goes non-finite (a profile ratio
  beyond the FP32 range) is solved again in FP64 (info.fallback);
* no solve loops without end: a breakdown counts as an iteration, and three
  breakdowns without progress end the column.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lattice, log

pytestmark = pytest.mark.gpu


def true_residual(U, C, M, alpha, S, eta, bc_t=-1):
    a6 = alpha[:, None, None, None, None, None]
    r = a6 * eta - oracle.apply(U, C, M, a6 * S, alpha=alpha, bc_t=bc_t)
    return float(np.linalg.norm(r) / np.linalg.norm(a6 * eta))


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_bicgstab_breakdown_restarts_with_random_shadow(precision):
    dims, M, r = (4, 4, 4, 4), 0.5, 1e-10
    log(f"test_bicgstab_breakdown_restarts_with_random_shadow {precision}")
    U = synth.free_gauge(dims)
    C = np.zeros(tuple(dims) + (12, 12), dtype=np.complex128)
    C[0, 0, 0, 0] = -(4.0 + M) * np.eye(12)
    alpha = np.ones(dims[0])
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols=2)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover_field(C)
        L.set_mass(M)
        L.set_alpha(alpha)
        S, cpp, info = L.solve(eta, r=r, precision=precision, max_iter=2000)
    log("  iters", [i["iters"] for i in info], "restarts", [i["restarts"] for i in info],
        "outer", [i["outer"] for i in info])
    for k in range(2):
        assert info[k]["status"] == 0
        assert info[k]["restarts"] >= 1
        assert true_residual(U, C, M, alpha, S[k], eta[k]) <= 1.0001 * r


@pytest.mark.parametrize("precision", ["f32", "f16"])
def test_nonfinite_inner_solve_falls_back_to_fp64(precision):
    dims, M, r = (6, 4, 4, 4), 0.5, 1e-10
    log(f"test_nonfinite_inner_solve_falls_back_to_fp64 {precision}")
    U = synth.gauge_su3(dims, 0.3, 11)
    C = oracle.clover(U, 1.6)
    alpha = np.ones(dims[0])
    alpha[-1] = 1e-40  # the hop ratio 1e40 into the last timeslice exceeds the FP32 range
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols=2)
    with lattice(dims, bc_t=0) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_alpha(alpha)
        S, cpp, info = L.solve(eta, r=r, precision=precision, max_iter=2000)
        S64, cpp64, info64 = L.solve(eta, r=r, precision="f64", max_iter=2000)
    log("  fallback", [i["fallback"] for i in info], "iters", [i["iters"] for i in info],
        "FP64 alone", [i["iters"] for i in info64])
    for k in range(2):
        assert info[k]["status"] == 0 and info[k]["fallback"] == 1
        assert info64[k]["fallback"] == 0
        assert true_residual(U, C, M, alpha, S[k], eta[k], bc_t=0) <= 1.0001 * r
        assert np.array_equal(S[k], S64[k])
