"""SAP+GCR on the GPU (the solver of the paper's light-quark iteration counts,
Table 1) against the oracle's SAP+GCR: the same iteration count with FP64
block solves, at most a few more with the FP32 ones, the oracle's residual of
the returned solution and its C_PP, with and without the light-quark
factorisation; invalid blockings are rejected."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lattice, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("alpha0", [0.0, 0.3])
def test_sap_gcr_vs_oracle(precision, alpha0):
    dims, block, M, r = (8, 4, 8, 4), (4, 2, 4, 2), 0.05, 1e-10
    log(f"test_sap_gcr_vs_oracle {precision} alpha0={alpha0}")
    U = synth.gauge_su3(dims, 0.4, 44)
    C = oracle.clover(U, 1.6)
    beta = synth.beta_cosh_paper(dims, alpha0)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))[3]
    S_or, info_or = oracle.solve_sap(U, C, M, eta, block, beta=beta, nkv=8, r=r)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_beta(beta)
        S, cpp, info = L.solve_sap(eta, block, r=r, nkv=8, precision=precision)
    log(f"  iterations GPU {info['iters']} oracle {info_or['iters']}, restarts {info['outer']}")
    assert info["status"] == 0
    if precision == "f64":
        assert abs(info["iters"] - info_or["iters"]) <= 1
    else:
        assert info["iters"] <= info_or["iters"] + 3
    bf = oracle.beta_field(dims, beta)[..., None, None]
    res = bf * eta - oracle.apply_beta(U, C, M, bf * S, beta)
    assert np.linalg.norm(res) / np.linalg.norm(bf * eta) <= 1.0001 * r
    np.testing.assert_allclose(cpp, oracle.cpp(S), rtol=1e-12)
    assert np.abs(cpp / oracle.cpp(S_or) - 1).max() < 1e-7


def test_sap_rejects_bad_blocks():
    import paper_1006_4028_amd as dp
    dims = (8, 4, 8, 4)
    with lattice(dims) as L:
        eta = synth.point_sources_12(dims, (0, 0, 0, 0))[0]
        for block in ((8, 2, 4, 2), (3, 2, 4, 2), (4, 4, 4, 2)):
            with pytest.raises(dp.DPError) as e:
                L.solve_sap(eta, block)
            assert e.value.code == -1


# One application of the preconditioner against the oracle's, element by
# element.  With FP32 block solves, blocks of at most 256 sites run the fused
# kernel (one launch per colour pass), blocks of up to 1536 sites its
# large-block variant; DP_SAP_FUSED=0, larger blocks and FP64 block solves
# take the launch-per-step path.  The FP32
# bound: each of the 5 x 2 passes rounds every residual and correction to
# FP32 (2^-24 relative) through 4 minimal-residual steps with O(10)-term
# sums, which stays within a few 1e-6 of the FP64 result in norm.
@pytest.mark.parametrize("dims,block", [((8, 4, 8, 4), (4, 2, 4, 2)),   # 64-site blocks, 16 of them
                                        ((8, 8, 8, 8), (4, 4, 4, 4)),   # 256 sites: every lane of the workgroup
                                        ((4, 4, 4, 8), (2, 2, 2, 2)),   # 16 sites: most lanes idle
                                        ((8, 6, 4, 4), (4, 3, 2, 2)),   # odd extent within a block
                                        ((16, 8, 8, 8), (8, 4, 4, 4)),  # 512 sites: the large-block kernel
                                        ((12, 12, 12, 12), (6, 6, 6, 6)),  # 1296 sites (the 48x24^3 blocking)
                                        ((16, 12, 8, 16), (8, 6, 4, 8)),   # 1536 sites: its largest block
                                        ((16, 16, 16, 8), (8, 8, 8, 4))])  # 2048 sites: launch per step
@pytest.mark.parametrize("path", ["fused", "steps", "f64"])
def test_sap_precondition_vs_oracle(dims, block, path, monkeypatch):
    log(f"test_sap_precondition_vs_oracle {dims} {block} {path}")
    monkeypatch.setenv("DP_SAP_FUSED", "0" if path == "steps" else "1")
    U = synth.gauge_su3(dims, 0.4, 45)
    C = oracle.clover(U, 1.6)
    M = 0.05
    beta = synth.beta_cosh_paper(dims, 0.3)
    r = synth.random_spinor(dims, 46)
    want = oracle.sap_apply(U, C, M, r, block, beta=beta)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_beta(beta)
        got = L.sap_precondition(r, block, precision="f64" if path == "f64" else "f32")
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    worst = np.abs(got - want).max() / np.abs(want).max()
    log(f"  relative error {err:.2e}, max {worst:.2e}")
    if path == "f64":
        assert err < 1e-12
    else:
        assert err < 1e-5 and worst < 1e-5


def test_sap_fused_matches_steps(monkeypatch):
    """The fused kernel and the launch-per-step path compute the same FP32
    block solves in different orders: they agree to FP32 rounding."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    log("test_sap_fused_matches_steps")
    U = synth.gauge_su3(dims, 0.4, 47)
    r = synth.random_spinor(dims, 48)
    out = {}
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.01)
        L.set_beta(synth.beta_cosh_paper(dims, 0.2))
        for path in ("1", "0"):
            monkeypatch.setenv("DP_SAP_FUSED", path)
            out[path] = L.sap_precondition(r, block, ncy=3, nmr=6)
    err = np.linalg.norm(out["1"] - out["0"]) / np.linalg.norm(out["0"])
    log(f"  fused vs steps {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("dims,block", [((8, 8, 8, 8), (4, 4, 4, 4)), ((12, 12, 12, 12), (6, 6, 6, 6))])
def test_sap_precondition_dirichlet_time(dims, block):
    """Dirichlet time boundary (bc_t = 0, the Schroedinger-functional hops):
    the hops across x0 = T-1 -> 0 drop in the block residual of both fused
    kernels, as in the oracle."""
    log(f"test_sap_precondition_dirichlet_time {dims} {block}")
    U = synth.gauge_su3(dims, 0.4, 49)
    C = oracle.clover(U, 1.6)
    M = 0.2
    r = synth.random_spinor(dims, 50)
    want = oracle.sap_apply(U, C, M, r, block, bc_t=0)
    with lattice(dims, bc_t=0) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        got = L.sap_precondition(r, block)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    worst = np.abs(got - want).max() / np.abs(want).max()
    log(f"  relative error {err:.2e}, max {worst:.2e}")
    assert err < 1e-5 and worst < 1e-5


def test_sap_precondition_full_size_32c64():
    """The preconditioner at the SAP study's full size and launch shape
    (64x32^3, 4^4 blocks, cosh factorisation alpha0 = 0.4, M = 0.05) against
    the oracle's, element by element over all 2.1 M sites."""
    cfg = synth.config("su3_32c64")
    dims = cfg["dims"]
    block = (4, 4, 4, 4)
    log("test_sap_precondition_full_size_32c64: fields")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    beta = synth.beta_cosh_paper(dims, 0.4)
    r = synth.random_spinor(dims, 51)
    log("  oracle")
    want = oracle.sap_apply(U, C, 0.05, r, block, beta=beta)
    del C
    log("  GPU")
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(cfg["csw"])
        L.set_mass(0.05)
        L.set_beta(beta)
        got = L.sap_precondition(r, block)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    worst = np.abs(got - want).max() / np.abs(want).max()
    log(f"  relative error {err:.2e}, max {worst:.2e}")
    assert err < 1e-5 and worst < 1e-5


def test_solve_sap_dev_matches_host():
    """The device-buffer SAP+GCR entry point gives bitwise the host variant's
    solution and C_PP (same kernels, same order); overlapping eta and S are
    rejected."""
    import torch
    import paper_1006_4028_amd as dp
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    log("test_solve_sap_dev_matches_host")
    U = synth.gauge_su3(dims, 0.4, 52)
    eta = synth.point_sources_12(dims, (1, 0, 0, 0))[5]
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.05)
        L.set_beta(synth.beta_cosh_paper(dims, 0.3))
        S, cpp, info = L.solve_sap(eta, block, r=1e-10, nkv=8)
        e_t = torch.from_numpy(np.ascontiguousarray(eta)).cuda()
        S_t = torch.zeros_like(e_t)
        cpp_d, info_d = L.solve_sap_dev(e_t, S_t, block, r=1e-10, nkv=8)
        assert info_d["iters"] == info["iters"]
        np.testing.assert_array_equal(S_t.cpu().numpy(), S)
        np.testing.assert_array_equal(cpp_d, cpp)
        with pytest.raises(dp.DPError) as e:
            L.solve_sap_dev(e_t, e_t, block, r=1e-10, nkv=8)
        assert e.value.code == -1


def test_sap_nonfinite_reports_and_recovers():
    """A time profile whose hop ratio (1e40) exceeds the FP32 range makes the
    FP32 block solves non-finite: GCR stops at the first non-finite norm with
    DP_ERR_NONFINITE, and the context solves normally afterwards (its vectors
    are assigned afresh, not scaled by zero)."""
    import paper_1006_4028_amd as dp
    dims, block = (8, 4, 8, 4), (4, 2, 4, 2)
    log("test_sap_nonfinite_reports_and_recovers")
    U = synth.gauge_su3(dims, 0.4, 53)
    C = oracle.clover(U, 1.6)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))[0]
    alpha = np.ones(dims[0])
    alpha[-1] = 1e-40
    with lattice(dims, bc_t=0) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.2)
        L.set_alpha(alpha)
        with pytest.raises(dp.DPError) as e:
            L.solve_sap(eta, block, r=1e-10, nkv=8)
        assert e.value.code == -6
        L.set_alpha(np.ones(dims[0]))
        S, cpp, info = L.solve_sap(eta, block, r=1e-10, nkv=8)
    assert info["status"] == 0
    res = eta - oracle.apply(U, C, 0.2, S, bc_t=0)
    assert np.linalg.norm(res) / np.linalg.norm(eta) <= 1.0001e-10


def test_sap_max_iter_returns_partial_solution():
    """Reaching max_iter reports DP_ERR_NOT_CONVERGED with the solution of the
    completed restart cycles, whose residual the oracle confirms is below
    the source's; the preconditioner entry point rejects a bad blocking."""
    import paper_1006_4028_amd as dp
    dims, block = (8, 4, 8, 4), (4, 2, 4, 2)
    log("test_sap_max_iter_returns_partial_solution")
    U = synth.gauge_su3(dims, 0.4, 54)
    C = oracle.clover(U, 1.6)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))[2]
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.05)
        S, cpp, info = L.solve_sap(eta, block, r=1e-12, nkv=2, max_iter=4, allow_unconverged=True)
        assert info["status"] == -4 and info["iters"] == 4
        res = np.linalg.norm(eta - oracle.apply(U, C, 0.05, S)) / np.linalg.norm(eta)
        log(f"  residual after 4 iterations {res:.2e} (GPU {info['true_res']:.2e})")
        assert res < 0.1 and abs(res / info["true_res"] - 1) < 1e-6
        with pytest.raises(dp.DPError) as e:
            L.sap_precondition(eta, (3, 2, 4, 2))
        assert e.value.code == -1
