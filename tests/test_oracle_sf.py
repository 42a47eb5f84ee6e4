"""Pin the oracle's Schroedinger-functional clover term and operator (the
formulation the closing remark of the heavy-quark section names, run there
with the exponential profile).  The interior lattice has T timeslices with
Dirichlet time boundaries; the two boundary timeslices carry fixed spatial
links and enter the interior only through the clover leaves (and, for the
boundary sources, through the backward time hop).

* periodic continuation: a padded lattice whose boundary timeslices are the
  periodic neighbours (the last and first timeslice) has the periodic clover
  in its interior; a boundary slice shifted by one fails;
* abelian boundary fields on a free interior: only the (0,k) leaves that touch
  a boundary differ from one, giving c_sw/4 sum_k sigma_0k (x) diag(sin theta_k)
  on the first interior timeslice and -c_sw/4 sum_k sigma_0k (x)
  diag(sin theta'_k) on the last one (theta_k = phi / L_k), zero in between;
  a wrong leaf orientation flips a sign, a direction mix-up swaps an L_k;
* the counterterm (ct_tilde - 1) on exactly the first and last timeslices;
* the operator equals the padded lattice's operator on fields that vanish on
  the boundaries.
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import GAMMA


def sigma(mu, nu):
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


def test_periodic_continuation():
    dims = (6, 4, 2, 4)
    U = synth.gauge_su3(dims, 0.7, seed=41)
    U_ext = np.concatenate([U[-1:], U, U[:1]], axis=0)
    np.testing.assert_allclose(oracle.sf_clover(U_ext, 1.6), oracle.clover(U, 1.6), atol=1e-14)
    # the boundary slices off by one: the first and last interior timeslices differ
    bad = np.concatenate([U[-2:-1], U, U[:1]], axis=0)
    d = np.abs(oracle.sf_clover(bad, 1.6) - oracle.clover(U, 1.6)).max(axis=(1, 2, 3, 4, 5))
    assert d[0] > 1e-3 and np.all(d[1:] < 1e-14)


def test_abelian_boundary_fields():
    dims = (5, 4, 6, 2)
    phi, phi_p = (-0.7, 0.2, 0.5), (0.9, -0.3, -0.6)
    csw, ct = 1.7, 1.25
    U_ext = synth.gauge_su3_sf(dims, 0.0, 0, phi, phi_p, interior_free=True)
    C = oracle.sf_clover(U_ext, csw, ct)
    first = np.zeros((12, 12), dtype=np.complex128)
    last = np.zeros((12, 12), dtype=np.complex128)
    for k in (1, 2, 3):
        first += csw / 4 * np.kron(sigma(0, k), np.diag(np.sin(np.array(phi) / dims[k])))
        last -= csw / 4 * np.kron(sigma(0, k), np.diag(np.sin(np.array(phi_p) / dims[k])))
    eye = (ct - 1.0) * np.eye(12)
    np.testing.assert_allclose(C[0], np.broadcast_to(first + eye, C[0].shape), atol=1e-14)
    np.testing.assert_allclose(C[-1], np.broadcast_to(last + eye, C[-1].shape), atol=1e-14)
    np.testing.assert_allclose(C[1:-1], 0.0, atol=1e-14)


def test_counterterm_only_next_to_the_boundaries():
    dims = (4, 2, 4, 2)
    U_ext = synth.gauge_su3_sf(dims, 0.6, 43, (0.1, 0.2, -0.3), (-0.4, 0.1, 0.3))
    d = oracle.sf_clover(U_ext, 1.3, 0.8) - oracle.sf_clover(U_ext, 1.3, 1.0)
    expect = np.zeros_like(d)
    expect[0] = expect[-1] = -0.2 * np.eye(12)
    np.testing.assert_allclose(d, expect, atol=1e-15)


@pytest.mark.parametrize("dagger", [False, True])
def test_operator_is_the_padded_operator_on_interior_fields(dagger):
    dims = (4, 4, 2, 2)
    U_ext = synth.gauge_su3_sf(dims, 0.6, 44, (0.3, -0.1, -0.2), (0.2, 0.2, -0.4))
    psi = synth.random_spinor(dims, 45)
    alpha = synth.alpha_exp(dims[0], 0.4)
    got = oracle.sf_apply(U_ext, 1.6, 0.3, psi, alpha=alpha, dagger=dagger)
    pad = np.zeros((dims[0] + 2,) + psi.shape[1:], dtype=np.complex128)
    pad[1:-1] = psi
    a_ext = np.concatenate([[alpha[0]], alpha, [alpha[-1]]])
    full = oracle.apply(U_ext, oracle.clover(U_ext, 1.6), 0.3, pad, alpha=a_ext, bc_t=0, dagger=dagger)
    np.testing.assert_allclose(got, full[1:-1], atol=1e-13)
