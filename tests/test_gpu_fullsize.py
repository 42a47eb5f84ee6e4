"""GPU results at the full workload sizes, checked against the oracle.

* 16^3 x 32 (heavy M = 0.5, c_sw = 1.6, 12 point-source columns): C_PP(t)
  per timeslice against the oracle's stored correlator (tests/golden,
  written by tests/golden/make_golden.py from oracle/ only), FP64 and mixed
  precision, alpha0 = 0.4 (eq. pbcalpha) within 1e-8 at every timeslice;
  alpha0 = 0 reported (the paper's loss of far timeslices under a global
  residual, heavy-quark section);
* 24^3 x 48 in the launch configuration bench.py times (12 columns, FP32
  inner): the oracle recomputes the true residual of sampled columns, and
  the C_PP of the 12 columns (their sum and each one) agrees with the
  oracle's stored correlator within 1e-8 at every timeslice;
* the full operator at 24^3 x 48 element by element against the oracle;
* 32^3 x 64 at the light mass M = 0.01 (CG on the normal equations, FP16
  storage, the symmetric exponential profile in both signs): the oracle
  recomputes the true residual of sampled columns and their C_PP, and the
  FP16 correlator of each column agrees per timeslice with the FP64 GPU solve
  and with the oracle's stored correlator (tests/golden).
"""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_common import lattice, log, max_rel

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cpp_su3_16c32_M0.5.txt")
GOLDEN_24C48 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cpp_su3_24c48_M0.5.txt")
GOLDEN_32C64 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cpp_su3_32c64_M0.01.txt")


def load_golden():
    return np.loadtxt(GOLDEN)[:, 1]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_16c32_cpp_against_oracle_golden(precision):
    import torch
    cfg = synth.config("su3_16c32")
    dims = cfg["dims"]
    log(f"test_16c32_cpp_against_oracle_golden {precision}")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    ref = load_golden()
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    e_t = torch.from_numpy(eta.reshape(12, -1)).cuda()
    errs = {}
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(cfg["csw"])
        L.set_mass(0.5)
        for a0 in (0.0, 0.4):
            L.set_alpha(synth.alpha_table("cosh", dims[0], a0))
            cpp, info = L.solve_dev(e_t, None, r=1e-11, precision=precision, ncols_group=12)
            assert all(i["status"] == 0 and i["true_res"] <= 1e-11 for i in info)
            errs[a0] = np.abs(cpp[0] / ref - 1)
            first = int(np.argmax(errs[a0] > 1e-8)) if np.any(errs[a0] > 1e-8) else None
            log(f"  alpha0={a0}: max per-timeslice rel err {errs[a0].max():.2e}, first t above 1e-8: {first}, "
                f"iters {[i['iters'] for i in info]}")
    assert errs[0.4].max() <= 1e-8
    # the preconditioned solve resolves the far timeslices at least as well
    assert errs[0.4][8:25].max() <= max(errs[0.0][8:25].max(), 1e-12)


def test_24c48_bench_configuration_true_residual():
    import torch
    cfg = synth.config("su3_24c48")
    dims, M = cfg["dims"], cfg["masses"][0]
    log("test_24c48_bench_configuration_true_residual")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    alpha = synth.alpha_table(cfg["profile"], dims[0], 0.4)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))
    e_t = torch.from_numpy(eta.reshape(12, -1)).cuda()
    S32 = torch.empty_like(e_t)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(cfg["csw"])
        L.set_mass(M)
        L.set_alpha(alpha)
        cpp32, info32 = L.solve_dev(e_t, S32, r=1e-11, precision="f32")
        cpp64, info64 = L.solve_dev(e_t, None, r=1e-11, precision="f64")
    S = S32.cpu().numpy().reshape((12,) + tuple(dims) + (4, 3))
    a6 = alpha[:, None, None, None, None, None]
    for c in (0, 7, 11):
        res = a6 * eta[c] - oracle.apply(U, C, M, a6 * S[c], alpha=alpha)
        tr = np.linalg.norm(res) / np.linalg.norm(a6 * eta[c])
        log(f"  column {c}: oracle true residual {tr:.3e}, GPU {info32[c]['true_res']:.3e}")
        assert tr <= 1.0001e-11
        # the correlator of the column equals the oracle's C_PP of the same S
        np.testing.assert_allclose(cpp32[c], oracle.cpp(S[c]), rtol=1e-12)
    err = np.abs(cpp32.sum(axis=0) / cpp64.sum(axis=0) - 1).max()
    log(f"  mixed vs FP64 C_PP max per-timeslice rel err {err:.2e}")
    assert err <= 1e-8
    # against the FP64 oracle's correlator of the same 12 columns (tests/golden,
    # written by make_golden.py from oracle/ only), every timeslice t = 0..47
    gold = np.loadtxt(GOLDEN_24C48)
    for name, cpp in (("mixed", cpp32), ("FP64", cpp64)):
        e = np.abs(cpp.sum(axis=0) / gold[:, 1] - 1)
        log(f"  {name} C_PP vs oracle: max per-timeslice rel err {e.max():.2e} (t = {int(np.argmax(e))})")
        assert e.max() <= 1e-8
        ec = np.abs(cpp / gold[:, 2:].T - 1).max()
        log(f"  {name} per-column C_PP vs oracle: max rel err {ec:.2e}")
        assert ec <= 1e-8


def test_24c48_operator_element_by_element():
    cfg = synth.config("su3_24c48")
    dims = cfg["dims"]
    log("test_24c48_operator_element_by_element")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    alpha = synth.alpha_table(cfg["profile"], dims[0], 0.4)
    psi = synth.random_spinor(dims, 99)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(cfg["csw"])
        L.set_mass(0.5)
        L.set_alpha(alpha)
        got = L.apply(psi, precond=True)
        got32 = L.apply(psi, precond=True, precision="f32")
    ref = oracle.apply(U, C, 0.5, psi, alpha=alpha)
    assert max_rel(got, ref) < 1e-13
    assert max_rel(got32, ref) < 1e-6


@pytest.mark.parametrize("alpha0", [0.1, -0.1])
def test_32c64_light_mass_cgnr_fp16(alpha0):
    cfg = synth.config("su3_32c64")
    dims, M, r = cfg["dims"], cfg["masses"][0], cfg["r"]
    log(f"test_32c64_light_mass_cgnr_fp16 alpha0={alpha0}")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    alpha = synth.alpha_table(cfg["profile"], dims[0], alpha0)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))[[0, 7]]
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(cfg["csw"])
        L.set_mass(M)
        L.set_alpha(alpha)
        S, cpp16, info = L.solve(eta, r=r, solver="cgnr", precision="f16", max_iter=20000)
        _, cpp64, info64 = L.solve(eta, r=r, solver="cgnr", precision="f64", max_iter=20000, want_S=False)
    log(f"  iters FP16 {[i['iters'] for i in info]}, FP64 {[i['iters'] for i in info64]}")
    a6 = alpha[:, None, None, None, None, None]
    for k in range(2):
        assert info[k]["status"] == 0 and info64[k]["status"] == 0
        res = a6 * eta[k] - oracle.apply(U, C, M, a6 * S[k], alpha=alpha)
        tr = np.linalg.norm(res) / np.linalg.norm(a6 * eta[k])
        log(f"  column {k}: oracle true residual {tr:.3e}, GPU {info[k]['true_res']:.3e}")
        assert tr <= 1.0001 * r
        np.testing.assert_allclose(cpp16[k], oracle.cpp(S[k]), rtol=1e-12)
        err = np.abs(cpp16[k] / cpp64[k] - 1).max()
        # The stopping norm weighs timeslice t by alpha(t)^2, so a residual r
        # bounds the error of S(t) relative to alpha(src)/alpha(t) times what
        # it bounds without preconditioning: the paper's light-quark profile
        # (alpha0 < 0 here, steepening the decay) gives up that factor at the
        # far timeslices.
        bound = 1e-8 * max(1.0, float(np.max(alpha[0] / alpha)))
        log(f"  FP16 vs FP64 C_PP max per-timeslice rel err {err:.2e} (bound {bound:.2e})")
        assert err <= bound
        # against the FP64 oracle's correlator of the same column (tests/golden;
        # the correlator does not depend on the profile the oracle solved with)
        gold = np.loadtxt(GOLDEN_32C64)[:, 2 + k]
        eg = np.abs(cpp16[k] / gold - 1)
        log(f"  column {k}: FP16 C_PP vs oracle max per-timeslice rel err {eg.max():.2e} (t = {int(np.argmax(eg))})")
        assert eg.max() <= bound


def test_32c64_light_quark_factorisation_iterations():
    """The paper's light-quark use (light-quark section, eqs. redefa, betaa):
    beta(y) = prod_mu cosh[alpha0 (y_mu - L_mu/2)] on the 32^3 x 64 workload,
    BiCGStab (FP32 inner) and CGNR (FP16 inner) for alpha0 in {0, 0.05, 0.1};
    every solve converges and the oracle recomputes its residual.  The
    iteration counts are reported (the paper's gains are for SAP+GCR on its
    dynamical ensembles; none is asserted here)."""
    import torch
    cfg = synth.config("su3_32c64")
    dims, M, r = cfg["dims"], cfg["masses"][0], cfg["r"]
    log("test_32c64_light_quark_factorisation_iterations")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    C = oracle.clover(U, cfg["csw"])
    eta = synth.point_sources_12(dims, (0, 0, 0, 0))[[0]]
    e_t = torch.from_numpy(eta.reshape(1, -1)).cuda()
    S_t = torch.empty_like(e_t)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(cfg["csw"])
        L.set_mass(M)
        for a0 in (0.0, 0.05, 0.1):
            beta = synth.beta_cosh_paper(dims, a0)
            L.set_beta(beta)
            for solver, prec in (("bicgstab", "f32"), ("cgnr", "f16")):
                cpp, info = L.solve_dev(e_t, S_t, r=r, solver=solver, precision=prec, max_iter=20000)
                S = S_t.cpu().numpy().reshape(eta.shape)[0]
                bf = oracle.beta_field(dims, beta)[..., None, None]
                res = bf * eta[0] - oracle.apply_beta(U, C, M, bf * S, beta)
                tr = np.linalg.norm(res) / np.linalg.norm(bf * eta[0])
                log(f"  alpha0={a0} {solver} {prec}: iters {info[0]['iters']}, oracle true residual {tr:.2e}")
                assert info[0]["status"] == 0 and tr <= 1.0001 * r
