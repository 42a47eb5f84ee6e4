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


@pytest.mark.parametrize("x0_src,profile", [(5, "exp"), (11, "exp"), (7, "cosh")])
def test_source_timeslice_shift(x0_src, profile):
    """A point source on timeslice x0_src of the free field.  Translation
    invariance fixes the propagator: S(x) = s(x0) S_closed((x0 - x0_src) mod T,
    x) with s = -1 for the sink timeslices the antiperiodic wrap separates
    from the source (x0 < x0_src).  The correlator indexed by t = (x0 - x0_src)
    mod T (the C_PP definition of the heavy-quark section, read for sources
    off the origin as the distance from the source timeslice) must then equal
    the closed form from the origin at every t.  The profile is measured from
    the source timeslice, as the served requests use it."""
    dims, M = (12, 4, 4, 4), 0.5
    T = dims[0]
    U = synth.free_gauge(dims)
    a = synth.alpha_table(profile, T, 0.4, x0_src)
    Sc = free_propagator_columns(dims, M)
    sign = np.where(np.arange(T) < x0_src, -1.0, 1.0)[:, None, None, None, None, None]
    S = []
    for c in range(12):
        eta = synth.point_source(dims, (x0_src, 0, 0, 0), c // 3, c % 3)
        Sk, info = oracle.solve(U, None, M, eta, alpha=a, r=1e-13)
        assert info["relres"] < 1e-12
        ref = sign * np.roll(Sc[c], x0_src, axis=0)
        np.testing.assert_allclose(Sk, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        S.append(Sk)
    S = np.stack(S)
    c_cf = free_cpp(dims, M)
    np.testing.assert_allclose(oracle.cpp(S, x0_src=x0_src), c_cf, rtol=1e-11)
    # the unshifted index puts the source's correlator at its lattice timeslice
    np.testing.assert_allclose(oracle.cpp(S, x0_src=0)[x0_src], c_cf[0], rtol=1e-11)
    # a subset of columns: C_PP sums over the given columns only
    np.testing.assert_allclose(oracle.cpp(S[:3], x0_src=x0_src),
                               -np.sum(np.abs(np.roll(Sc[:3], 0, axis=1)) ** 2, axis=(0, 2, 3, 4, 5, 6)),
                               rtol=1e-11)
