"""Pin the oracle's SAP+GCR (the solver of the paper's Table 1).

* the colour-restricted operator is the direct sum of the Dirichlet block
  operators (blocks of one colour never touch);
* with the block solves run to convergence, one SAP cycle leaves no residual
  on the blocks solved last;
* GCR preconditioned by SAP reaches the LAPACK solution (4^4, 2^4 blocks),
  the BiCGStab solution of an interacting beta-preconditioned system for any
  restart length, and the closed-form free propagator.
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import free_propagator_columns
from test_oracle_dense import dense


def colours(dims, block):
    x = np.indices(dims)
    b = [x[mu] // block[mu] for mu in range(4)]
    return (sum(b) % 2), np.ravel_multi_index(b, [dims[mu] // block[mu] for mu in range(4)])


def test_colour_restriction_is_the_block_direct_sum():
    dims, block, M = (4, 4, 8, 4), (2, 2, 4, 2), 0.2
    U = synth.gauge_su3(dims, 0.7, 41)
    C = oracle.clover(U, 1.6)
    beta = tuple(np.exp(np.random.default_rng(2).uniform(-0.5, 0.5, L)) for L in dims)
    col, blk = colours(dims, block)
    psi = synth.random_spinor(dims, 5)
    m0 = (col == 0)[..., None, None]
    whole = oracle.apply_beta(U, C, M, psi * m0, beta) * m0
    for b in np.unique(blk[col == 0])[:3]:
        mb = (blk == b)[..., None, None]
        one = oracle.apply_beta(U, C, M, psi * mb, beta) * mb
        np.testing.assert_allclose(whole * mb, one, rtol=0, atol=1e-13 * np.abs(one).max())


def test_converged_block_solves_leave_no_residual_on_the_last_colour():
    dims, block, M = (4, 4, 4, 4), (2, 2, 2, 2), 0.3
    U = synth.gauge_su3(dims, 0.5, 42)
    C = oracle.clover(U, 1.6)
    r = synth.random_spinor(dims, 6)
    psi = oracle.sap_apply(U, C, M, r, block, ncy=1, nmr=400)
    col, _ = colours(dims, block)
    res = r - oracle.apply(U, C, M, psi)
    m1 = (col == 1)[..., None, None]
    assert np.linalg.norm(res * m1) < 1e-10 * np.linalg.norm(r)
    assert np.linalg.norm(res * ~m1) > 1e-3 * np.linalg.norm(r)  # colour 0 was solved before colour 1 changed psi


def test_gcr_reaches_the_lapack_solution():
    dims, block, M = (4, 4, 4, 4), (2, 2, 2, 2), 0.1
    U = synth.gauge_su3(dims, 1.0, 43)
    C = oracle.clover(U, 1.6)
    eta = synth.random_spinor(dims, 7)
    D = dense(lambda p: oracle.apply(U, C, M, p), dims)
    ref = np.linalg.solve(D, eta.reshape(-1)).reshape(eta.shape)
    S, info = oracle.solve_sap(U, C, M, eta, block, r=1e-12)
    assert info["relres_prec"] < 1e-12
    np.testing.assert_allclose(S, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("nkv", [3, 16])
def test_gcr_matches_bicgstab_with_light_quark_factorisation(nkv):
    dims, block, M = (8, 4, 8, 4), (4, 2, 4, 2), 0.05
    U = synth.gauge_su3(dims, 0.4, 44)
    C = oracle.clover(U, 1.6)
    beta = synth.beta_cosh_paper(dims, 0.2)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))[3]
    S0, i0 = oracle.solve(U, C, M, eta, beta=beta, r=1e-13)
    S1, i1 = oracle.solve_sap(U, C, M, eta, block, beta=beta, nkv=nkv, r=1e-12)
    assert i1["relres_prec"] < 1e-12
    np.testing.assert_allclose(S1, S0, rtol=0, atol=1e-10 * np.abs(S0).max())
    assert i1["iters"] < i0["iters"]


def test_free_propagator():
    dims, block, M = (8, 4, 4, 4), (4, 2, 2, 2), 0.2
    U = synth.free_gauge(dims)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    Sc = free_propagator_columns(dims, M)
    beta = synth.beta_cosh_paper(dims, 0.3)
    for c in (0, 8):
        S, info = oracle.solve_sap(U, None, M, eta[c], block, beta=beta, r=1e-13)
        np.testing.assert_allclose(S, Sc[c], rtol=0, atol=1e-11 * np.abs(Sc[c]).max())
