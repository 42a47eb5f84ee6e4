"""GPU solves against the FP64 oracle and the closed form.

* free field 8^3 x 16 (Wilson, M = 0.5, alpha = exp(0.4 t), 12 point sources
  at the origin, FP64 BiCGStab to r = 1e-11): S and C_PP against the
  momentum-space closed form;
* interacting fields with clover on small lattices: S and C_PP against the
  oracle's solve, for BiCGStab and CGNR in FP64, FP32 and FP16 inner
  precision, alpha0 = 0 and 0.4;
* the true residual of every returned solution recomputed by the oracle;
* batch invariance: each right-hand side gives the same bits alone and in a
  batch.
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import free_cpp, free_propagator_columns
from gpu_common import lattice, log, rel_err

pytestmark = pytest.mark.gpu


def true_residual(U, C, M, alpha, S, eta, bc_t=-1):
    """Oracle recomputation of |eta' - D'S'| / |eta'| with S' = alpha S."""
    a6 = alpha[:, None, None, None, None, None]
    Sp, ep = a6 * S, a6 * eta
    r = ep - oracle.apply(U, C, M, Sp, alpha=alpha, bc_t=bc_t)
    return float(np.linalg.norm(r) / np.linalg.norm(ep))


def test_free_field_closed_form():
    cfg = synth.config("free_8c16")
    dims, M = cfg["dims"], cfg["masses"][0]
    log(f"test_free_field_closed_form dims={dims}")
    alpha = synth.alpha_exp(dims[0], 0.4)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    Sc = free_propagator_columns(dims, M)
    with lattice(dims) as L:
        L.set_mass(M)
        L.set_alpha(alpha)
        S, cpp, info = L.solve(eta, r=1e-11, ncols_group=12)
    log("  iters", [i["iters"] for i in info], "true_res", max(i["true_res"] for i in info))
    assert all(i["status"] == 0 and i["true_res"] <= 1e-11 for i in info)
    for c in range(12):
        assert np.abs(S[c] - Sc[c]).max() < 1e-10 * np.abs(Sc[c]).max()
    ref = free_cpp(dims, M)
    err = np.abs(cpp[0] / ref - 1)
    log("  max per-timeslice C_PP rel err", err.max())
    assert err.max() < 1e-8
    U = synth.free_gauge(dims)
    for c in (0, 7):
        assert true_residual(U, None, M, alpha, S[c], eta[c]) <= 1.0001e-11


@pytest.mark.parametrize("solver,precision", [("bicgstab", "f64"), ("bicgstab", "f32"), ("bicgstab", "f16"),
                                              ("cgnr", "f64"), ("cgnr", "f32"), ("cgnr", "f16")])
@pytest.mark.parametrize("alpha0", [0.0, 0.4])
def test_interacting_solve_vs_oracle(solver, precision, alpha0):
    dims, M, r = (12, 4, 6, 4), 0.5, 1e-11  # Vh = 576: two full tiles and a ragged one
    log(f"test_interacting_solve_vs_oracle {solver} {precision} alpha0={alpha0}")
    U = synth.gauge_su3(dims, 0.3, 77)
    C = oracle.clover(U, 1.6)
    alpha = synth.alpha_exp(dims[0], alpha0)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    cols = [0, 5, 11]
    S_or = np.stack([oracle.solve(U, C, M, eta[c], alpha=alpha, r=1e-14)[0] for c in cols])
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_alpha(alpha)
        S, cpp, info = L.solve(eta[cols], r=r, solver=solver, precision=precision, max_iter=20000)
    log("  iters", [i["iters"] for i in info], "outer", [i["outer"] for i in info],
        "true_res", [f"{i['true_res']:.2e}" for i in info])
    for k, c in enumerate(cols):
        assert info[k]["status"] == 0
        tr = true_residual(U, C, M, alpha, S[k], eta[c])
        assert tr <= 1.0001 * r, tr
        assert rel_err(S[k], S_or[k]) < 50 * r
        cpp_or = oracle.cpp(S_or[k])
        assert np.abs(cpp[k] / cpp_or - 1).max() < 1e-8


def test_batch_invariance():
    """A right-hand side gives the same bits alone and inside a batch."""
    dims = (8, 4, 4, 6)
    log("test_batch_invariance")
    U = synth.gauge_su3(dims, 0.4, 5)
    alpha = synth.alpha_exp(dims[0], 0.2)
    eta = synth.random_spinor(dims, 21, nrhs=5)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.3)
        L.set_alpha(alpha)
        for precision in ("f64", "f32"):
            S_all, cpp_all, info_all = L.solve(eta, r=1e-10, precision=precision)
            for k in (0, 3):
                S1, cpp1, info1 = L.solve(eta[k], r=1e-10, precision=precision)
                assert info1[0]["iters"] == info_all[k]["iters"]
                assert np.array_equal(S1[0], S_all[k]), precision
                assert np.array_equal(cpp1[0], cpp_all[k])


def test_c2_shape_smoke_and_residual():
    """16^3 x 32 interacting field as in the 16^3 x 32 workload (the paper's
    periodic-time profile, eq. pbcalpha): two columns, FP64 and mixed, the
    true residual recomputed by the oracle and the C_PP of the two within
    1e-8 per timeslice."""
    cfg = synth.config("su3_16c32")
    dims = cfg["dims"]
    log(f"test_c2_shape dims={dims}")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    alpha = synth.alpha_table(cfg["profile"], dims[0], 0.4)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols=2)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(cfg["csw"])
        L.set_mass(0.5)
        L.set_alpha(alpha)
        S64, c64, i64 = L.solve(eta, r=1e-11)
        S32, c32, i32 = L.solve(eta, r=1e-11, precision="f32")
    log("  f64 iters", [i["iters"] for i in i64], "f32 iters", [i["iters"] for i in i32])
    for k in range(2):
        assert true_residual(U, C, 0.5, alpha, S64[k], eta[k]) <= 1.0001e-11
        assert true_residual(U, C, 0.5, alpha, S32[k], eta[k]) <= 1.0001e-11
        assert np.abs(c32[k] / c64[k] - 1).max() < 1e-8


def test_error_codes():
    import paper_1006_4028_amd as dp
    dims = (4, 4, 4, 4)
    with lattice(dims) as L:
        with pytest.raises(dp.DPError) as e:
            L.set_alpha(np.array([1.0, -1.0, 1.0, 1.0]))
        assert e.value.code == -1
        with pytest.raises(dp.DPError):
            L.solve(synth.random_spinor(dims, 1), r=-1.0)
        eta = synth.random_spinor(dims, 2)
        eta[0, 0, 0, 0, 0, 0] = np.nan
        with pytest.raises(dp.DPError) as e:
            L.solve(eta, r=1e-10)
        assert e.value.code == -6
        L.set_mass(0.1)
        S, cpp, info = L.solve(synth.random_spinor(dims, 3), r=1e-12, max_iter=1, allow_unconverged=True)
        assert info[0]["status"] == -4
    with pytest.raises(dp.DPError):
        dp.Lattice((4, 4, 3, 4))


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
@pytest.mark.parametrize("alpha0", [0.1, -0.1])
def test_light_mass_cgnr_vs_oracle(precision, alpha0):
    """The light-quark workload's solver (CG on the normal equations, FP16
    storage with per-site scales for the inner solve) at M = 0.01 with the
    symmetric exponential profile in both signs, on a small lattice."""
    dims, M, r = (8, 4, 4, 6), 0.01, 1e-10
    log(f"test_light_mass_cgnr_vs_oracle {precision} alpha0={alpha0}")
    U = synth.gauge_su3(dims, 0.2, 3264)
    C = oracle.clover(U, 1.6)
    alpha = synth.alpha_exp_sym(dims[0], alpha0)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols=2)
    S_or = np.stack([oracle.solve(U, C, M, eta[c], alpha=alpha, r=1e-13, solver="cgnr")[0] for c in range(2)])
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_alpha(alpha)
        S, cpp, info = L.solve(eta, r=r, solver="cgnr", precision=precision, max_iter=50000)
    log("  iters", [i["iters"] for i in info], "outer", [i["outer"] for i in info])
    for k in range(2):
        assert info[k]["status"] == 0
        assert true_residual(U, C, M, alpha, S[k], eta[k]) <= 1.0001 * r
        assert np.abs(cpp[k] / oracle.cpp(S_or[k]) - 1).max() < 1e-7


@pytest.mark.parametrize("solver", ["cgnr", "bicgstab"])
def test_fp16_point_source_long_support(solver):
    """FP16 storage on a lattice large enough that a point source's Krylov
    vectors keep sites holding only rounding residues of cancellations for
    many iterations (32 x 16^3).  Those residues shrink by about the FP32
    epsilon per operator application; the per-site scale of such a site must
    not overflow when it falls below the smallest normal float (regression:
    the CGNR solve went non-finite at its third iteration)."""
    dims, M, r = (32, 16, 16, 16), 0.01, 1e-10
    log(f"test_fp16_point_source_long_support {solver}")
    U = synth.gauge_su3(dims, 0.2, 3264)
    C = oracle.clover(U, 1.6)
    alpha = synth.alpha_exp_sym(dims[0], 0.1)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols=1)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_alpha(alpha)
        S, cpp, info = L.solve(eta, r=r, solver=solver, precision="f16", max_iter=20000)
    log("  iters", info[0]["iters"], "outer", info[0]["outer"])
    assert info[0]["status"] == 0
    assert np.isfinite(S).all()
    assert true_residual(U, C, M, alpha, S[0], eta[0]) <= 1.0001 * r


@pytest.mark.parametrize("solver,precision", [("bicgstab", "f64"), ("bicgstab", "f32"), ("cgnr", "f16")])
def test_light_quark_factorisation_solve_vs_oracle(solver, precision):
    """Solves with beta(y) = prod_mu cosh[alpha0 (y_mu - L_mu/2)] (the paper's
    eq. betaa in the convention S' = beta S): the restored S and C_PP (the
    restoration precedes the contraction, light-quark section) equal the
    oracle's, and the oracle recomputes the residual of the preconditioned
    system from the returned S.  Changing the spatial profiles while a batch
    is open is refused."""
    dims, M, r = (8, 4, 6, 4), 0.1, 1e-10
    log(f"test_light_quark_factorisation_solve_vs_oracle {solver} {precision}")
    U = synth.gauge_su3(dims, 0.3, 77)
    C = oracle.clover(U, 1.6)
    beta = synth.beta_cosh_paper(dims, 0.3)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols=2)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_beta(beta)
        S, cpp, info = L.solve(eta, r=r, solver=solver, precision=precision, max_iter=50000)
        import paper_1006_4028_amd as dp
        b = dp.Batch(L, 2, "f32")
        with pytest.raises(dp.DPError) as e:
            L.set_alpha_space(None, None, None)
        assert e.value.code == -7
        b.close()
        L.set_alpha_space(None, None, None)
    bf = oracle.beta_field(dims, beta)[..., None, None]
    log("  iters", [i["iters"] for i in info])
    for k in range(2):
        assert info[k]["status"] == 0
        S_or, _ = oracle.solve(U, C, M, eta[k], beta=beta, r=1e-13)
        res = bf * eta[k] - oracle.apply_beta(U, C, M, bf * S[k], beta)
        assert np.linalg.norm(res) / np.linalg.norm(bf * eta[k]) <= 1.0001 * r
        np.testing.assert_allclose(cpp[k], oracle.cpp(S[k]), rtol=1e-12)
        assert np.abs(cpp[k] / oracle.cpp(S_or) - 1).max() < 1e-7
