"""Pin the oracle's light-quark preconditioning (eqs. redefa, betaa, redefcovs).

beta(y) = prod_mu alpha_mu(y_mu) with one profile per direction.  The oracle
applies D' = beta (D+M) beta^-1 literally (orc_apply_beta) and through the
modified covariant derivatives in all four directions with the boundary
rule continued in each direction (orc_apply_modified4); they must agree for
any profiles and any extension values (the method is an exact similarity),
and both must agree with beta_field * (D+M)(psi / beta_field) built here
from the unpreconditioned oracle operator.  The restored solution of the
beta-preconditioned system equals the closed-form free propagator and the
unpreconditioned solve, and the adjoint satisfies D'(beta)^+ =
gamma5 D'(1/beta) gamma5.
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import GAMMA5, free_propagator_columns


def g5(psi):
    return np.einsum("ij,...jc->...ic", GAMMA5, psi)


def random_profiles(dims, seed):
    rng = np.random.default_rng(seed)
    return tuple(np.exp(rng.uniform(-1.0, 1.0, L)) for L in dims)


@pytest.fixture(scope="module")
def field():
    dims = (4, 4, 6, 4)
    U = synth.gauge_su3(dims, 0.8, seed=21)
    C = oracle.clover(U, 1.6)
    return dims, U, C


@pytest.mark.parametrize("bc_t", [-1, 1])
def test_modified_covariant_derivatives_equal_similarity(field, bc_t):
    dims, U, C = field
    M = 0.15
    beta = random_profiles(dims, 3)
    bf = oracle.beta_field(dims, beta)[..., None, None]
    psi = synth.random_spinor(dims, 4)
    lit = oracle.apply_beta(U, C, M, psi, beta, bc_t=bc_t)
    ref = bf * oracle.apply(U, C, M, psi / bf, bc_t=bc_t)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(lit, ref, rtol=0, atol=1e-13 * scale)
    for ext in ([1.0] * 8, [3.0, 0.2, 7.0, 0.5, 0.01, 40.0, 1.3, 2.2]):
        mod = oracle.apply_modified4(U, C, M, psi, beta, ext, bc_t=bc_t)
        np.testing.assert_allclose(mod, ref, rtol=0, atol=1e-12 * scale)
    # the time-only profile is the heavy-quark alpha of eq. redeft
    a0 = (beta[0], None, None, None)
    np.testing.assert_allclose(oracle.apply_beta(U, C, M, psi, a0, bc_t=bc_t),
                               oracle.apply(U, C, M, psi, alpha=beta[0], bc_t=bc_t), rtol=0, atol=1e-13 * scale)


def test_adjoint_and_gamma5_relation(field):
    dims, U, C = field
    M = 0.3
    beta = random_profiles(dims, 7)
    inv = tuple(1.0 / b for b in beta)
    phi, psi = synth.random_spinor(dims, 8), synth.random_spinor(dims, 9)
    Dpsi = oracle.apply_beta(U, C, M, psi, beta)
    Ddphi = oracle.apply_beta(U, C, M, phi, beta, dagger=True)
    lhs, rhs = np.vdot(phi, Dpsi), np.vdot(Ddphi, psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    alt = g5(oracle.apply_beta(U, C, M, g5(phi), inv))
    np.testing.assert_allclose(Ddphi, alt, rtol=0, atol=1e-13 * np.abs(alt).max())


@pytest.mark.parametrize("alpha0", [0.2, 0.5])
def test_free_propagator_with_light_quark_profile(alpha0):
    """S' = beta S_closed with the paper's four-direction cosh factorisation,
    and the restored S equals the closed form."""
    dims, M = (8, 4, 6, 4), 0.3
    U = synth.free_gauge(dims)
    beta = synth.beta_cosh_paper(dims, alpha0)
    bf = oracle.beta_field(dims, beta)[..., None, None]
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    Sc = free_propagator_columns(dims, M)
    for c in (1, 9):
        for solver in ("bicgstab", "cgnr"):
            S, Sp, info = oracle.solve(U, None, M, eta[c], beta=beta, r=1e-13, solver=solver, return_prec=True)
            np.testing.assert_allclose(S, Sc[c], rtol=0, atol=1e-12 * np.abs(Sc[c]).max())
            np.testing.assert_allclose(Sp, bf * Sc[c], rtol=0, atol=1e-11 * np.abs(Sp).max())


def test_interacting_solve_restores_unpreconditioned():
    dims, M = (4, 4, 6, 4), 0.2
    U = synth.gauge_su3(dims, 0.5, seed=33)
    C = oracle.clover(U, 1.6)
    beta = synth.beta_cosh_paper(dims, 0.3)
    eta = synth.random_spinor(dims, 12)
    S0, i0 = oracle.solve(U, C, M, eta, r=1e-13)
    for solver in ("bicgstab", "cgnr"):
        S1, i1 = oracle.solve(U, C, M, eta, beta=beta, r=1e-13, solver=solver)
        assert i1["relres"] < 1e-11
        np.testing.assert_allclose(S1, S0, rtol=0, atol=1e-11 * np.abs(S0).max())
