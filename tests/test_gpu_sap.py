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
