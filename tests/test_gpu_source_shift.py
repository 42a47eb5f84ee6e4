"""Sources off the origin: the correlator index t = (x0 - x0_src) mod T of the
C_PP definition (heavy-quark section), and the point sources of
dp_point_sources.

* free field: point sources on timeslice x0_src written by dp_point_sources,
  solved with the profile measured from the source; S equals the
  translated closed form (sign -1 across the antiperiodic wrap) and C_PP the
  closed form from the origin, per timeslice;
* interacting field with clover: GPU solves at x0_src != 0 against the
  oracle's solve of the same source and the oracle's C_PP of it, per
  timeslice;
* a batch request at x0_src != 0: its C_PP equals the oracle's C_PP of the
  returned S, and the oracle's solve.
"""
import numpy as np
import pytest

import oracle
import synth
from closed_form import free_cpp, free_propagator_columns
from gpu_common import lattice, log

pytestmark = pytest.mark.gpu


def test_point_sources_match_the_definition():
    import torch
    dims = (6, 4, 2, 4)
    log("test_point_sources_match_the_definition")
    with lattice(dims) as L:
        for site, c0, n in (((0, 0, 0, 0), 0, 12), ((5, 3, 1, 2), 4, 3), ((2, 0, 1, 3), 11, 1)):
            got = L.point_sources(site, c0, n).cpu().numpy().reshape((n,) + dims + (4, 3))
            ref = np.stack([synth.point_source(dims, site, (c0 + j) // 3, (c0 + j) % 3) for j in range(n)])
            assert np.array_equal(got, ref), (site, c0, n)
        import paper_1006_4028_amd as dp
        for bad in (((0, 0, 0, 0), 10, 3), ((6, 0, 0, 0), 0, 1), ((0, 0, 0, 0), -1, 2)):
            with pytest.raises(dp.DPError):
                L.point_sources(bad[0], bad[1], bad[2], out=torch.empty((max(bad[2], 1), L.V * 12),
                                                                        dtype=torch.complex128, device="cuda"))


@pytest.mark.parametrize("x0_src", [5, 15])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_free_field_source_shift_closed_form(x0_src, precision):
    import torch
    cfg = synth.config("free_8c16")
    dims, M = cfg["dims"], cfg["masses"][0]
    T = dims[0]
    log(f"test_free_field_source_shift_closed_form x0_src={x0_src} {precision}")
    alpha = synth.alpha_exp(T, 0.4, x0_src)
    Sc = free_propagator_columns(dims, M)
    sign = np.where(np.arange(T) < x0_src, -1.0, 1.0)[:, None, None, None, None, None]
    with lattice(dims) as L:
        L.set_mass(M)
        L.set_alpha(alpha)
        eta_t = L.point_sources((x0_src, 0, 0, 0))
        S_t = torch.empty_like(eta_t)
        cpp, info = L.solve_dev(eta_t, S_t, r=1e-11, precision=precision, x0_src=x0_src, ncols_group=12)
    assert all(i["status"] == 0 and i["true_res"] <= 1e-11 for i in info)
    S = S_t.cpu().numpy().reshape((12,) + tuple(dims) + (4, 3))
    for c in range(12):
        ref = sign * np.roll(Sc[c], x0_src, axis=0)
        assert np.abs(S[c] - ref).max() < 1e-10 * np.abs(ref).max(), c
    err = np.abs(cpp[0] / free_cpp(dims, M) - 1)
    log(f"  max per-timeslice C_PP rel err {err.max():.2e}")
    assert err.max() < 1e-8


@pytest.mark.parametrize("x0_src", [3, 7])
def test_interacting_source_shift_vs_oracle(x0_src):
    dims, M, r = (8, 4, 4, 6), 0.5, 1e-11
    T = dims[0]
    log(f"test_interacting_source_shift_vs_oracle x0_src={x0_src}")
    U = synth.gauge_su3(dims, 0.3, 81)
    C = oracle.clover(U, 1.6)
    alpha = synth.alpha_table("cosh", T, 0.4, x0_src)
    eta = synth.point_sources_12(dims, (x0_src, 0, 0, 0))
    cols = [0, 4, 11]
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(M)
        L.set_alpha(alpha)
        for precision in ("f64", "f32"):
            S, cpp, info = L.solve(eta[cols], r=r, precision=precision, x0_src=x0_src)
            for k, c in enumerate(cols):
                assert info[k]["status"] == 0
                S_or, _ = oracle.solve(U, C, M, eta[c], alpha=alpha, r=1e-14)
                c_or = oracle.cpp(S_or, x0_src=x0_src)
                e = np.abs(cpp[k] / c_or - 1).max()
                log(f"  {precision} column {c}: max per-timeslice C_PP rel err vs oracle {e:.2e}")
                assert e <= 1e-8
                # the GPU's own contraction of its S, by the oracle's definition
                np.testing.assert_allclose(cpp[k], oracle.cpp(S[k], x0_src=x0_src), rtol=1e-12)


def test_batch_request_off_the_origin_vs_oracle():
    import torch
    import paper_1006_4028_amd as dp
    from paper_1006_4028_amd.serve import point_columns, profile
    dims, r = (8, 4, 4, 6), 1e-10
    log("test_batch_request_off_the_origin_vs_oracle")
    U = synth.gauge_su3(dims, 0.4, 17)
    C = oracle.clover(U, 1.6)
    reqs = [dict(M=0.2, a0=0.1, x0=6, cols=2), dict(M=0.5, a0=0.4, x0=3, cols=1)]
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        with dp.Batch(L, 4, "f32") as B:
            for k, q in enumerate(reqs):
                eta = point_columns(dims, q["x0"], q["cols"])
                q["eta"] = eta
                q["S_t"] = torch.zeros(q["cols"], eta[0].size, dtype=torch.complex128, device="cuda")
                q["slots"] = B.admit(torch.from_numpy(eta.reshape(q["cols"], -1)).cuda(), q["S_t"], M=q["M"],
                                     alpha=profile(dims[0], q["a0"], q["x0"]), r=r, x0_src=q["x0"], tag=k)
            got = []
            while B.status()["running"] or B.status()["done"]:
                B.step(3)
                got += B.harvest()
    for res in got:
        q = reqs[res["tag"]]
        c = q["slots"].index(res["slot"])
        S_b = q["S_t"].cpu().numpy().reshape((q["cols"],) + dims + (4, 3))[c]
        np.testing.assert_allclose(res["cpp"], oracle.cpp(S_b, x0_src=q["x0"]), rtol=1e-12)
        alpha = profile(dims[0], q["a0"], q["x0"])
        S_or, _ = oracle.solve(U, C, q["M"], q["eta"][c], alpha=alpha, r=1e-14)
        e = np.abs(res["cpp"] / oracle.cpp(S_or, x0_src=q["x0"]) - 1).max()
        log(f"  request {res['tag']} column {c} x0={q['x0']}: C_PP vs oracle {e:.2e}")
        assert e <= 1e-7
