"""Pin the oracle with dense linear algebra on tiny lattices.

* the modified time derivatives and the boundary rule eq. redeftbc give
  exactly alpha (D+M) alpha^-1 (eq. linsysprec; the method is an exact
  similarity, introduction), whatever values alpha takes outside [0, T);
* the spectra of D'+M and D+M coincide;
* gamma5-hermiticity of D+M (with clover), and the adjoint the oracle applies
  equals the conjugate transpose;
* BiCGStab and CGNR reach the LAPACK (numpy.linalg.solve) solution.

2^4 cannot tell psi(x+mu) from psi(x-mu); 4^4 can.
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import GAMMA5


def dense(op, dims):
    V = synth.volume(dims)
    n = V * 12
    A = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = op(e.reshape(tuple(dims) + (4, 3))).reshape(-1)
        e[j] = 0.0
    return A


def g5_full(V):
    return np.kron(np.eye(V), np.kron(GAMMA5, np.eye(3)))


@pytest.fixture(scope="module", params=[(2, 2, 2, 2), (4, 4, 4, 4)], ids=["2^4", "4^4"])
def setup(request):
    dims = request.param
    U = synth.gauge_su3(dims, 1.0, seed=11)
    C = oracle.clover(U, 1.6)
    rng = np.random.default_rng(5)
    alpha = np.exp(rng.uniform(-1.5, 1.5, dims[0]))
    return dims, U, C, alpha


@pytest.mark.parametrize("bc_t", [-1, 1])
def test_modified_derivatives_equal_similarity(setup, bc_t):
    dims, U, C, alpha = setup
    if dims[0] > 2 and bc_t == 1:
        pytest.skip("covered by the 2^4 case and the antiperiodic 4^4 case")
    M = 0.2
    D = dense(lambda p: oracle.apply(U, C, M, p, bc_t=bc_t), dims)
    Dp = dense(lambda p: oracle.apply_modified(U, C, M, p, alpha, 3.7, 0.21, bc_t=bc_t), dims)
    a = np.repeat(alpha, synth.volume(dims) // dims[0] * 12)
    ref = (a[:, None] * D) / a[None, :]
    np.testing.assert_allclose(Dp, ref, atol=1e-13 * np.abs(ref).max())
    # the extension of alpha beyond the lattice drops out (eq. redeftbc)
    psi = synth.random_spinor(dims, 3)
    o1 = oracle.apply_modified(U, C, M, psi, alpha, 1.0, 1.0, bc_t=bc_t)
    o2 = oracle.apply_modified(U, C, M, psi, alpha, 123.0, 1e-3, bc_t=bc_t)
    np.testing.assert_allclose(o1, o2, atol=1e-12 * np.abs(o1).max())
    # the literal form agrees with the modified form
    o3 = oracle.apply(U, C, M, psi, alpha=alpha, bc_t=bc_t)
    np.testing.assert_allclose(o3, o1, atol=1e-12 * np.abs(o1).max())
    if dims[0] == 2:
        from scipy.optimize import linear_sum_assignment
        ev, evp = np.linalg.eigvals(D), np.linalg.eigvals(Dp)
        dist = np.abs(ev[:, None] - evp[None, :])
        rows, cols = linear_sum_assignment(dist)
        assert dist[rows, cols].max() < 1e-9


def test_gamma5_hermiticity_and_adjoint(setup):
    dims, U, C, alpha = setup
    M = 0.1
    V = synth.volume(dims)
    D = dense(lambda p: oracle.apply(U, C, M, p), dims)
    G5 = g5_full(V)
    H = G5 @ D
    np.testing.assert_allclose(H, H.conj().T, atol=1e-13)
    Dp = dense(lambda p: oracle.apply(U, C, M, p, alpha=alpha), dims)
    Dpd = dense(lambda p: oracle.apply(U, C, M, p, alpha=alpha, dagger=True), dims)
    np.testing.assert_allclose(Dpd, Dp.conj().T, atol=1e-12 * np.abs(Dp).max())
    # D'(alpha)^+ = gamma5 D'(1/alpha) gamma5
    Dinv = dense(lambda p: oracle.apply(U, C, M, p, alpha=1.0 / alpha), dims)
    np.testing.assert_allclose(Dpd, G5 @ Dinv @ G5, atol=1e-12 * np.abs(Dp).max())


def test_clover_structure(setup):
    dims, U, C, _ = setup
    Cf = C.reshape(-1, 12, 12)
    np.testing.assert_allclose(Cf, np.conj(np.swapaxes(Cf, 1, 2)), atol=1e-14)
    g5 = np.kron(GAMMA5, np.eye(3))
    np.testing.assert_allclose(g5 @ Cf - Cf @ g5, 0, atol=1e-14)
    assert np.abs(Cf).max() > 0.1
    C0 = oracle.clover(synth.free_gauge(dims), 1.6)
    assert np.abs(C0).max() == 0.0


@pytest.mark.parametrize("solver", ["bicgstab", "cgnr"])
def test_solvers_reach_lapack_solution(setup, solver):
    dims, U, C, alpha = setup
    M = 0.3
    Dp = dense(lambda p: oracle.apply(U, C, M, p, alpha=alpha), dims)
    eta = synth.random_spinor(dims, 9)
    a = np.repeat(alpha, synth.volume(dims) // dims[0] * 12)
    x_lu = np.linalg.solve(Dp, a * eta.reshape(-1)) / a  # S = S'/alpha
    S, info = oracle.solve(U, C, M, eta, alpha=alpha, r=1e-13, solver=solver)
    assert info["relres_prec"] < 1e-12
    cond = np.linalg.cond(Dp)
    np.testing.assert_allclose(S.reshape(-1), x_lu, atol=10 * cond * 1e-13 * np.abs(x_lu).max())
