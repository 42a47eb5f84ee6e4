"""Pin the oracle to the closed-form free Wilson propagator.

The momentum-space form (tests/closed_form.py) is derived from the operator
definition independently of the oracle's position-space code: it pins the
hop term, the gamma basis, the fermion boundary condition, the mass
normalisation, the alpha redefinition S' = alpha S with its restoration, and
the correlator C_PP(y0) = -sum tr[S^+ S] (section on heavy quarks).
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import free_cpp, free_propagator_columns, free_propagator_spin


@pytest.mark.parametrize("bc_t", [-1, 1])
@pytest.mark.parametrize("dims", [(8, 4, 4, 4), (6, 2, 4, 2)])
def test_free_propagator_unpreconditioned(dims, bc_t):
    M = 0.5
    U = synth.free_gauge(dims)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    Sc = free_propagator_columns(dims, M, bc_t)
    for c in (0, 4, 11):
        S, info = oracle.solve(U, None, M, eta[c], r=1e-13, bc_t=bc_t)
        assert info["relres"] < 1e-12
        np.testing.assert_allclose(S, Sc[c], rtol=0, atol=1e-13)


@pytest.mark.parametrize("profile,alpha0", [("exp", 0.4), ("cosh", 0.4), ("exp_sym", 0.3)])
def test_free_propagator_preconditioned(profile, alpha0):
    """S' = alpha S_closed, and the restored S equals S_closed (eq. redeft,
    eq. linsysprec and restoration)."""
    dims, M = (12, 4, 4, 4), 0.5
    U = synth.free_gauge(dims)
    a = synth.alpha_table(profile, dims[0], alpha0)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    Sc = free_propagator_columns(dims, M)
    for c in (2, 7):
        S, Sp, info = oracle.solve(U, None, M, eta[c], alpha=a, r=1e-13, return_prec=True)
        np.testing.assert_allclose(S, Sc[c], rtol=0, atol=1e-13 * np.abs(Sc[c]).max())
        np.testing.assert_allclose(Sp, a[:, None, None, None, None, None] * Sc[c], rtol=0,
                                   atol=1e-12 * np.abs(Sp).max())


def test_free_cpp_c1_workload():
    """Free field 8^3 x 16, M = 0.5, alpha = exp(0.4 t), 12 point sources at the
    origin: the restored correlator equals the closed form at every timeslice,
    relative error per timeslice (not only the global norm)."""
    cfg = synth.config("free_8c16")
    dims, M = cfg["dims"], cfg["masses"][0]
    U = synth.free_gauge(dims)
    a = synth.alpha_exp(dims[0], 0.4)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    S = np.stack([oracle.solve(U, None, M, eta[c], alpha=a, r=1e-13)[0] for c in range(12)])
    c_or = oracle.cpp(S)
    c_cf = free_cpp(dims, M)
    assert np.all(c_cf < 0)
    np.testing.assert_allclose(c_or, c_cf, rtol=1e-10)
    # the same columns, built in closed form, give the same correlator via the oracle's C_PP
    np.testing.assert_allclose(oracle.cpp(free_propagator_columns(dims, M)), c_cf, rtol=1e-13)


def test_free_cpp_decay_rate():
    """At zero spatial momentum the free pole is exp(E) = 1 + M; C_PP sums all
    spatial momenta and so decays at large t as exp(-2 E t) with E = ln(1+M)."""
    dims, M = (64, 2, 2, 2), 0.5
    c = free_cpp(dims, M)
    # on L = 2 spatial momenta are 0 and pi: the pi modes are much heavier
    meff = np.log(c[10:20] / c[11:21])
    np.testing.assert_allclose(meff, 2 * np.log1p(M), rtol=1e-6)
    U = synth.free_gauge(dims)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    S = oracle.solve(U, None, M, eta[0], alpha=synth.alpha_exp(64, 0.4), r=1e-13)[0]
    cs = oracle.cpp(S)
    np.testing.assert_allclose(np.log(cs[10:20] / cs[11:21]), 2 * np.log1p(M), rtol=1e-6)


def test_closed_form_solves_the_oracle_equation():
    """Cross-pin in the other direction: applying the oracle's D+M to the closed
    form returns the point source."""
    dims, M = (8, 4, 2, 4), 0.3
    U = synth.free_gauge(dims)
    Sc = free_propagator_columns(dims, M, ncols=12)
    for c in (1, 9):
        eta = oracle.apply(U, None, M, Sc[c])
        ref = synth.point_source(dims, (0, 0, 0, 0), c // 3, c % 3)
        np.testing.assert_allclose(eta, ref, atol=1e-14)


def test_spin_propagator_symmetry():
    """gamma5-hermiticity in the closed form itself: S(x)^+ = gamma5 S(-x) gamma5
    holds for periodic time (a sanity check of tests/closed_form.py)."""
    from closed_form import GAMMA5
    dims = (4, 4, 4, 4)
    Ss = free_propagator_spin(dims, 0.2, bc_t=1)
    neg = Ss[(-np.arange(4)) % 4][:, (-np.arange(4)) % 4][:, :, (-np.arange(4)) % 4][:, :, :, (-np.arange(4)) % 4]
    lhs = np.conj(np.swapaxes(Ss, -1, -2))
    rhs = GAMMA5 @ neg @ GAMMA5
    np.testing.assert_allclose(lhs, rhs, atol=1e-14)
