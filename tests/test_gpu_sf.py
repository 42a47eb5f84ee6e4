"""GPU parity of the Schroedinger-functional operator and its boundary
sources against the oracle (the formulation of the closing remark of the
heavy-quark section): interior links and the boundary links enter through
dp_set_gauge_sf, the clover term is built on the padded lattice and carries
the counterterm (ct_tilde - 1) next to the boundaries, and the time hops stop
at the boundaries (bc_t = 0)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lattice, log, max_rel, oracle_schur

pytestmark = pytest.mark.gpu

PHI, PHI_P = (-0.6, 0.1, 0.5), (0.8, -0.3, -0.5)


def sf_case(dims, seed, eps=0.6):
    return synth.gauge_su3_sf(dims, eps, seed, PHI, PHI_P)


@pytest.mark.parametrize("dims", [(6, 4, 6, 4), (8, 4, 4, 4)])
def test_sf_operator(dims):
    """Full operator, Schur operator and adjoints in FP64, FP32 and FP16
    storage, with the distance-preconditioning profile on; first with the
    counterterm alone (c_sw = 0), then with the clover term."""
    log(f"test_sf_operator dims={dims}")
    U_ext = sf_case(dims, 60 + dims[2])
    U = U_ext[1:-1]
    ct, M = 1.3, 0.4
    alpha = synth.alpha_exp(dims[0], 0.4)
    psi = synth.random_spinor(dims, 61)
    with lattice(dims, bc_t=0) as L:
        L.set_gauge_sf(U_ext, ct)
        L.set_mass(M)
        L.set_alpha(alpha)
        for csw in (0.0, 1.6):
            if csw:
                L.set_clover(csw)
            C = oracle.sf_clover(U_ext, csw, ct)
            for dagger in (False, True):
                ref = oracle.sf_apply(U_ext, csw, M, psi, alpha=alpha, ct_tilde=ct, dagger=dagger)
                assert max_rel(L.apply(psi, precond=True, dagger=dagger), ref) < 1e-13, (csw, dagger)
                refs = oracle_schur(oracle, U, C, M, psi, alpha, bc_t=0, dagger=dagger)
                assert max_rel(L.apply(psi, precond=True, schur=True, dagger=dagger), refs) < 1e-12
                for precision, tol in (("f32", 2e-6), ("f16", 3e-3)):
                    e = max_rel(L.apply(psi, precond=True, schur=True, dagger=dagger, precision=precision), refs)
                    log(f"  csw={csw} {precision} dagger={dagger} max-element err {e:.2e}")
                    assert e < tol


def wall_sources_oracle(U_ext, ncols=12, side=0):
    """The boundary sources from the oracle's operator on the padded lattice:
    minus its action on a field that is e_c on the boundary (x0 = 0 for side
    0, x0 = T + 1 for side 1) and zero elsewhere, restricted to the interior
    (only the time hop out of the boundary-adjacent interior timeslice sees
    the boundary)."""
    Tp = U_ext.shape[0]
    out = []
    for c in range(ncols):
        phi = np.zeros(U_ext.shape[:4] + (4, 3), dtype=np.complex128)
        phi[0 if side == 0 else Tp - 1, ..., c // 3, c % 3] = 1.0
        out.append(-oracle.apply(U_ext, None, 0.0, phi, bc_t=0)[1:Tp - 1])
    return np.stack(out)


def test_sf_wall_sources():
    import paper_1006_4028_amd as dp
    dims = (6, 4, 2, 6)
    log("test_sf_wall_sources")
    U_ext = sf_case(dims, 62)
    ref = wall_sources_oracle(U_ext)
    ref1 = wall_sources_oracle(U_ext, side=1)
    assert np.abs(ref[:, 1:]).max() == 0.0 and np.abs(ref[:, 0]).max() > 0.1
    assert np.abs(ref1[:, :-1]).max() == 0.0 and np.abs(ref1[:, -1]).max() > 0.1
    with lattice(dims, bc_t=0) as L:
        with pytest.raises(dp.DPError):
            L.sf_wall_sources()  # no boundary links yet
        L.set_gauge_sf(U_ext, 1.0)
        got = L.sf_wall_sources().cpu().numpy().reshape(ref.shape)
        assert np.abs(got - ref).max() < 1e-15
        got1 = L.sf_wall_sources(side=1).cpu().numpy().reshape(ref.shape)
        assert np.abs(got1 - ref1).max() < 1e-15
        part = L.sf_wall_sources(c0=5, ncols=4).cpu().numpy().reshape((4,) + ref.shape[1:])
        assert np.array_equal(part, got[5:9])
        part1 = L.sf_wall_sources(c0=2, ncols=3, side=1).cpu().numpy().reshape((3,) + ref.shape[1:])
        assert np.array_equal(part1, got1[2:5])
        with pytest.raises(dp.DPError):
            L.sf_wall_sources(side=2)
        L.set_gauge(U_ext[1:-1])  # periodic-style links clear the boundary state
        with pytest.raises(dp.DPError):
            L.sf_wall_sources()
    with lattice(dims, bc_t=-1) as L:
        with pytest.raises(dp.DPError):
            L.set_gauge_sf(U_ext, 1.0)


def test_sf_far_boundary_correlator():
    """Sources on the x0 = T + 1 boundary: the correlator decays from the last
    interior timeslice towards the first; with the reversed exponential
    profile alpha = exp(0.5 (T - 1 - x0)) at r = 1e-11 it matches the
    oracle's solve per timeslice (interior 4^3 x 16, random field, M = 0.5,
    c_sw = 1.6, ct_tilde = 1.1)."""
    dims, M, csw, ct = (16, 4, 4, 4), 0.5, 1.6, 1.1
    log("test_sf_far_boundary_correlator")
    U_ext = sf_case(dims, 64, eps=0.3)
    C = oracle.sf_clover(U_ext, csw, ct)
    eta = wall_sources_oracle(U_ext, 6, side=1)
    alpha = synth.alpha_exp(dims[0], 0.5)[::-1].copy()
    exact = oracle.cpp(np.stack([oracle.solve(U_ext[1:-1], C, M, eta[c], alpha=alpha, r=1e-13, bc_t=0)[0]
                                 for c in range(6)]))
    with lattice(dims, bc_t=0) as L:
        L.set_gauge_sf(U_ext, ct)
        L.set_clover(csw)
        L.set_mass(M)
        L.set_alpha(alpha)
        eta_t = L.sf_wall_sources(ncols=6, side=1)
        cpp, info = L.solve_dev(eta_t, None, r=1e-11, precision="f32", ncols_group=6)
    err = np.abs(cpp[0] / exact - 1)
    log(f"  |C| first/last {abs(exact[0]):.2e} / {abs(exact[-1]):.2e}, max rel err {err.max():.2e}")
    assert all(i["status"] == 0 for i in info)
    assert np.all(np.diff(np.abs(exact)) > 0)  # grows towards the source boundary
    assert err.max() < 1e-8


def test_sf_boundary_correlator_loose_residue():
    """The boundary-to-bulk correlator (sum over the interior timeslice of
    |S|^2, the quantity C_PP reports) from the wall sources: with the
    profile and r = 1e-11 it matches the oracle's solve (r = 1e-13) per
    timeslice; at the loose residue 1e-6 the
    unpreconditioned solve is wrong at the far timeslices, while the
    exponential profile (end of the heavy-quark section) restored by
    eq. backcorrection stays right everywhere.  Interior 4^3 x 32 with a
    random gauge field, M = 0.5, c_sw = 1.6, ct_tilde = 1.1, alpha0 = 0.5."""
    dims, M, csw, ct = (32, 4, 4, 4), 0.5, 1.6, 1.1
    log("test_sf_boundary_correlator_loose_residue")
    U_ext = sf_case(dims, 63, eps=0.3)
    C = oracle.sf_clover(U_ext, csw, ct)
    eta = wall_sources_oracle(U_ext, 6)  # columns 6..11 are the negatives of 0..5
    alpha = synth.alpha_exp(dims[0], 0.5)
    exact = oracle.cpp(np.stack([oracle.solve(U_ext[1:-1], C, M, eta[c], alpha=alpha, r=1e-13, bc_t=0)[0]
                                 for c in range(6)]))
    with lattice(dims, bc_t=0) as L:
        L.set_gauge_sf(U_ext, ct)
        L.set_clover(csw)
        L.set_mass(M)
        eta_t = L.sf_wall_sources(ncols=6)
        assert np.abs(eta_t.cpu().numpy().reshape(eta.shape) - eta).max() < 1e-15
        L.set_alpha(alpha)
        c_tight, i_tight = L.solve_dev(eta_t, None, r=1e-11, precision="f64", ncols_group=6)
        c_prec, _ = L.solve_dev(eta_t, None, r=1e-6, precision="f32", ncols_group=6)
        L.set_alpha(np.ones(dims[0]))
        c_plain, _ = L.solve_dev(eta_t, None, r=1e-6, precision="f32", ncols_group=6)
    e_tight = np.abs(c_tight[0] / exact - 1)
    e_plain = np.abs(c_plain[0] / exact - 1)
    e_prec = np.abs(c_prec[0] / exact - 1)
    for k in range(0, dims[0], 3):
        log(f"  {k:2d}  {abs(exact[k]):.3e}  {e_tight[k]:.1e}  {e_plain[k]:.3e}  {e_prec[k]:.3e}")
    assert all(i["status"] == 0 for i in i_tight)
    assert np.all(np.diff(np.abs(exact)) < 0)  # decays over the whole extent
    assert e_tight.max() < 1e-8
    assert e_plain[-4:].max() > 1e-2
    assert e_prec.max() < 1e-4
