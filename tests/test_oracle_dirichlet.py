"""Pin the oracle's Dirichlet time boundary (bc_t = 0), the fermion boundary
of the Schroedinger functional with zero boundary fields (the paper used its
preconditioning there with the exponential profile, heavy-quark section).

* the operator is linear in the sign of the hops across the time boundary,
  so D(bc 0) = (D(bc +1) + D(bc -1)) / 2 exactly, with clover and alpha;
* the modified time derivatives with the boundary rule give the similarity
  for any extension of alpha (nothing crosses the boundary);
* gamma5-hermiticity; BiCGStab and CGNR reach the LAPACK solution;
* the free correlator from a source on the first timeslice decays over the
  whole time extent (no backward-propagating part).
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import GAMMA5
from test_oracle_dense import dense


@pytest.fixture(scope="module")
def field():
    dims = (6, 4, 4, 4)
    U = synth.gauge_su3(dims, 0.7, 51)
    return dims, U, oracle.clover(U, 1.6)


def test_dirichlet_is_the_average_of_the_two_signs(field):
    dims, U, C = field
    alpha = synth.alpha_exp(dims[0], 0.3)
    psi = synth.random_spinor(dims, 1)
    for dagger in (False, True):
        d0 = oracle.apply(U, C, 0.2, psi, alpha=alpha, bc_t=0, dagger=dagger)
        dp = oracle.apply(U, C, 0.2, psi, alpha=alpha, bc_t=1, dagger=dagger)
        dm = oracle.apply(U, C, 0.2, psi, alpha=alpha, bc_t=-1, dagger=dagger)
        np.testing.assert_allclose(d0, 0.5 * (dp + dm), rtol=0, atol=1e-13 * np.abs(d0).max())
        assert np.abs(d0 - dp).max() > 1e-3 * np.abs(d0).max()


def test_modified_derivatives_and_similarity(field):
    dims, U, C = field
    alpha = np.exp(np.random.default_rng(3).uniform(-1, 1, dims[0]))
    psi = synth.random_spinor(dims, 2)
    lit = oracle.apply(U, C, 0.1, psi, alpha=alpha, bc_t=0)
    for ext in ((1.0, 1.0), (50.0, 0.02)):
        mod = oracle.apply_modified(U, C, 0.1, psi, alpha, ext[0], ext[1], bc_t=0)
        np.testing.assert_allclose(mod, lit, rtol=0, atol=1e-12 * np.abs(lit).max())


def test_gamma5_hermiticity_and_lapack():
    dims = (4, 2, 2, 2)
    U = synth.gauge_su3(dims, 1.0, 52)
    C = oracle.clover(U, 1.6)
    D = dense(lambda p: oracle.apply(U, C, 0.1, p, bc_t=0), dims)
    G5 = np.kron(np.eye(synth.volume(dims)), np.kron(GAMMA5, np.eye(3)))
    H = G5 @ D
    np.testing.assert_allclose(H, H.conj().T, atol=1e-13)
    eta = synth.random_spinor(dims, 3)
    ref = np.linalg.solve(D, eta.reshape(-1)).reshape(eta.shape)
    for solver in ("bicgstab", "cgnr"):
        S, info = oracle.solve(U, C, 0.1, eta, r=1e-13, solver=solver, bc_t=0)
        np.testing.assert_allclose(S, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_free_correlator_decays_over_the_whole_extent():
    dims, M = (16, 4, 4, 4), 0.2
    U = synth.free_gauge(dims)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    S = np.stack([oracle.solve(U, None, M, eta[c], r=1e-13, bc_t=0)[0] for c in range(12)])
    c = -oracle.cpp(S)
    assert np.all(c > 0)
    assert np.all(np.diff(c) < 0)
    # with the periodic boundary the correlator turns back up at the far end
    Sp = np.stack([oracle.solve(U, None, M, eta[k], r=1e-13, bc_t=-1)[0] for k in range(12)])
    cp = -oracle.cpp(Sp)
    assert cp[-1] > cp[dims[0] // 2]


def test_dirichlet_equals_zero_padded_periodic_operator(field):
    """An independent construction: the lattice embedded between two extra
    timeslices on which the field vanishes, the periodic operator applied on
    the larger lattice and the result restricted to the original slices."""
    dims, U, C = field
    T = dims[0]
    ext = (T + 2,) + dims[1:]
    Ue = np.empty(ext + (4, 3, 3), dtype=np.complex128)
    Ue[1:T + 1] = U
    Ue[0] = Ue[T + 1] = synth.free_gauge((1,) + dims[1:])[0]
    Ce = np.zeros(ext + (12, 12), dtype=np.complex128)
    Ce[1:T + 1] = C
    psi = synth.random_spinor(dims, 4)
    pe = np.zeros(ext + (4, 3), dtype=np.complex128)
    pe[1:T + 1] = psi
    for bc in (-1, 1):
        out = oracle.apply(Ue, Ce, 0.2, pe, bc_t=bc)[1:T + 1]
        np.testing.assert_allclose(oracle.apply(U, C, 0.2, psi, bc_t=0), out, rtol=0, atol=1e-13 * np.abs(out).max())
