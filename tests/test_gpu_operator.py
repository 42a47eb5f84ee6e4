"""GPU parity of the operator kernels against the FP64 oracle, element by element.

The alpha-hop kernel (hop term of D' with the modified time derivatives,
heavy-quark section), its clover epilogues, the Schur operator of the
even-odd reduction, the adjoint, and the FP32 / FP16-storage variants.
Lattices span several 256-site tiles and end in a ragged tail.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lattice, log, max_rel, oracle_hop, oracle_schur, parity_mask

pytestmark = pytest.mark.gpu

DIMS = [(8, 4, 4, 4), (6, 4, 6, 4), (4, 6, 2, 8)]  # Vh = 256, 288 (ragged), 192


def setup_field(dims, seed, csw=1.6, eps=0.6):
    U = synth.gauge_su3(dims, eps, seed)
    rng = np.random.default_rng(seed)
    alpha = np.exp(rng.uniform(-1.0, 1.0, dims[0]))
    return U, oracle.clover(U, csw), alpha


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("bc_t", [-1, 1, 0])
def test_hop_only(dims, bc_t):
    log(f"test_hop_only dims={dims} bc_t={bc_t}")
    U, _, alpha = setup_field(dims, 100 + dims[1])
    psi = synth.random_spinor(dims, 7)
    with lattice(dims, bc_t) as L:
        L.set_gauge(U)
        L.set_mass(0.3)
        L.set_alpha(alpha)
        for precond in (False, True):
            for dagger in (False, True):
                got = L.apply(psi, precond=precond, dagger=dagger, hop_only=True)
                a = alpha if precond else None
                if dagger:
                    full = oracle.apply(U, None, 0.3, psi, alpha=a, bc_t=bc_t, dagger=True)
                    ref = full - 4.3 * psi
                else:
                    ref = oracle_hop(oracle, U, None, 0.3, psi, a, bc_t)
                assert max_rel(got, ref) < 1e-13, (precond, dagger)


@pytest.mark.parametrize("dims", DIMS)
def test_full_operator_with_clover(dims):
    log(f"test_full_operator_with_clover dims={dims}")
    U, C, alpha = setup_field(dims, 200 + dims[2])
    psi = synth.random_spinor(dims, 8)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.5)
        L.set_alpha(alpha)
        for precond in (False, True):
            for dagger in (False, True):
                got = L.apply(psi, precond=precond, dagger=dagger)
                ref = oracle.apply(U, C, 0.5, psi, alpha=alpha if precond else None, dagger=dagger)
                assert max_rel(got, ref) < 1e-13, (precond, dagger)


def test_clover_field_input_and_rejection():
    dims = (4, 4, 4, 4)
    log("test_clover_field_input_and_rejection")
    U, C, alpha = setup_field(dims, 5)
    psi = synth.random_spinor(dims, 9)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover_field(C)
        L.set_mass(0.2)
        L.set_alpha(alpha)
        got = L.apply(psi, precond=True)
        assert max_rel(got, oracle.apply(U, C, 0.2, psi, alpha=alpha)) < 1e-13
        bad = C.copy()
        bad[..., 0, 7] += 0.5  # mixes the chiralities
        import paper_1006_4028_amd as dp
        with pytest.raises(dp.DPError):
            L.set_clover_field(bad)


@pytest.mark.parametrize("dims", DIMS[:2])
def test_schur_operator(dims):
    log(f"test_schur_operator dims={dims}")
    U, C, alpha = setup_field(dims, 300 + dims[0])
    psi = synth.random_spinor(dims, 10)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.05)
        L.set_alpha(alpha)
        got = L.apply(psi, precond=True, schur=True)
        ref = oracle_schur(oracle, U, C, 0.05, psi, alpha)
        assert max_rel(got, ref) < 1e-12
        got_dag = L.apply(psi, precond=True, schur=True, dagger=True)
        assert max_rel(got_dag, oracle_schur(oracle, U, C, 0.05, psi, alpha, dagger=True)) < 1e-12
        # adjoint: <phi, Mhat psi> = <Mhat^+ phi, psi> on the even sites
        phi = synth.random_spinor(dims, 11)
        got_d = L.apply(phi, precond=True, schur=True, dagger=True)
        even = (parity_mask(dims) == 0)[..., None, None]
        lhs = np.vdot(phi * even, ref)
        rhs = np.vdot(got_d, psi * even)
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)


@pytest.mark.parametrize("precision,tol", [("f32", 2e-6), ("f16", 3e-3)])
def test_inner_precision_kernels(precision, tol):
    dims = (8, 4, 6, 4)
    log(f"test_inner_precision_kernels {precision}")
    U, C, _ = setup_field(dims, 400)
    alpha = synth.alpha_exp(dims[0], 0.4)
    psi = synth.random_spinor(dims, 12)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.5)
        L.set_alpha(alpha)
        for schur in (False, True):
            for dagger in (False, True):
                got = L.apply(psi, precond=True, schur=schur, dagger=dagger, precision=precision)
                if schur:
                    ref = oracle_schur(oracle, U, C, 0.5, psi, alpha, dagger=dagger)
                else:
                    ref = oracle.apply(U, C, 0.5, psi, alpha=alpha, dagger=dagger)
                e = max_rel(got, ref)
                log(f"  {precision} schur={schur} dagger={dagger} max-element err {e:.2e}")
                assert e < tol


@pytest.mark.parametrize("precision,nrhs", [("f64", 5), ("f32", 5), ("f16", 5), ("f32", 13), ("f32", 2)])
def test_apply_dev_multi_rhs_matches_per_column(precision, nrhs):
    """dp_apply_dev runs the multi-RHS kernels (every right-hand side a slot);
    each column must equal the one-slot dp_apply of that column bitwise (the
    slot arithmetic does not depend on the batch), for the full operator, the
    Schur operator and their adjoints; the per-launch timing samples match
    the launch counts.  13 FP32 columns take two passes of the shared-tile
    workgroup (7 waves, the last one idle in the second pass).  The lattice
    has 1536 sites per timeslice and parity: 24 chunks of 64 sites, three in
    every XCD's slab, so the chunk boundaries, the slab boundaries and the
    neighbours across them are all exercised."""
    import torch
    dims = (4, 16, 12, 16)
    log(f"test_apply_dev_multi_rhs_matches_per_column {precision} nrhs={nrhs}")
    U, _, alpha = setup_field(dims, 31)
    psi = synth.random_spinor(dims, 8, nrhs=nrhs)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.2)
        L.set_alpha(alpha)
        in_t = torch.from_numpy(psi.reshape(nrhs, -1)).cuda()
        out_t = torch.empty_like(in_t)
        for schur in (False, True):
            for dagger in (False, True):
                L.set_timing(True)
                L.apply_dev(in_t, out_t, precond=True, dagger=dagger, schur=schur, precision=precision)
                stats = L.timing()
                for name, st in stats.items():
                    assert len(L.timing_samples(name)) == st["launches"]
                L.set_timing(False)
                got = out_t.cpu().numpy().reshape(psi.shape)
                for k in range(nrhs):
                    ref = L.apply(psi[k], precond=True, dagger=dagger, schur=schur, precision=precision)
                    assert np.array_equal(got[k], ref), (schur, dagger, k)
        with pytest.raises(Exception):
            L.apply_dev(in_t, in_t, precond=True)


@pytest.mark.parametrize("dims", DIMS)
def test_light_quark_factorisation_operator(dims):
    """beta(y) = prod_mu a_mu(y_mu) (eqs. redefa, betaa, redefcovs): the full
    operator, the Schur operator and their adjoints against the oracle's
    literal beta (D+M) beta^-1, in FP64, FP32 and FP16 storage; with the
    preconditioning flag off the spatial profiles must not act."""
    log(f"test_light_quark_factorisation_operator dims={dims}")
    U, C, _ = setup_field(dims, 500 + dims[2])
    rng = np.random.default_rng(dims[1])
    beta = tuple(np.exp(rng.uniform(-0.7, 0.7, L)) for L in dims)
    psi = synth.random_spinor(dims, 13)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.25)
        L.set_beta(beta)
        for dagger in (False, True):
            ref = oracle.apply_beta(U, C, 0.25, psi, beta, dagger=dagger)
            assert max_rel(L.apply(psi, precond=True, dagger=dagger), ref) < 1e-12
            refs = oracle_schur(oracle, U, C, 0.25, psi, beta, dagger=dagger)
            assert max_rel(L.apply(psi, precond=True, schur=True, dagger=dagger), refs) < 1e-12
            for precision, tol in (("f32", 2e-6), ("f16", 3e-3)):
                e = max_rel(L.apply(psi, precond=True, schur=True, dagger=dagger, precision=precision), refs)
                log(f"  {precision} schur dagger={dagger} max-element err {e:.2e}")
                assert e < tol
        plain = oracle.apply(U, C, 0.25, psi)
        assert max_rel(L.apply(psi, precond=False), plain) < 1e-12


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-6), ("f16", 3e-3)])
def test_dirichlet_time_boundary_operator(precision, tol):
    """The Dirichlet time boundary (bc_t = 0): full and Schur operators and
    their adjoints against the oracle, every storage precision."""
    dims = (8, 4, 6, 4)
    log(f"test_dirichlet_time_boundary_operator {precision}")
    U, C, alpha = setup_field(dims, 600)
    psi = synth.random_spinor(dims, 14)
    with lattice(dims, bc_t=0) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.3)
        L.set_alpha(alpha)
        for dagger in (False, True):
            ref = oracle.apply(U, C, 0.3, psi, alpha=alpha, bc_t=0, dagger=dagger)
            assert max_rel(L.apply(psi, precond=True, dagger=dagger, precision=precision), ref) < tol
            refs = oracle_schur(oracle, U, C, 0.3, psi, alpha, bc_t=0, dagger=dagger)
            assert max_rel(L.apply(psi, precond=True, schur=True, dagger=dagger, precision=precision), refs) < tol
