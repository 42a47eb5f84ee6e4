"""Continuous batching on the GPU: right-hand sides with different masses,
profiles and source timeslices enter and leave a running batch; every result
equals the same right-hand side solved alone (bit for bit) and satisfies the
stopping rule when its residual is recomputed by the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lattice, log

pytestmark = pytest.mark.gpu

DIMS = (8, 4, 4, 6)


def solo(L, eta, M, alpha, x0, r, precision):
    L.set_mass(M)
    L.set_alpha(alpha)
    S, cpp, info = L.solve(eta, r=r, precision=precision, x0_src=x0)
    return S[0], cpp[0], info[0]


@pytest.mark.parametrize("precision", ["f64", "f32", "f16"])
def test_batch_join_and_leave_matches_solo(precision):
    import torch
    import paper_1006_4028_amd as dp
    from paper_1006_4028_amd.serve import point_columns, profile
    log(f"test_batch_join_and_leave_matches_solo {precision}")
    U = synth.gauge_su3(DIMS, 0.4, 17)
    C = oracle.clover(U, 1.6)
    r = 1e-10
    reqs = [dict(M=0.5, a0=0.4, x0=0, cols=3), dict(M=0.05, a0=0.0, x0=3, cols=2), dict(M=0.2, a0=0.1, x0=6, cols=1)]
    with lattice(DIMS) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        got = {}
        with dp.Batch(L, 5, precision) as B:
            def admit(k):
                q = reqs[k]
                eta = point_columns(DIMS, q["x0"], q["cols"])
                S_t = torch.zeros(q["cols"], eta[0].size, dtype=torch.complex128, device="cuda")
                slots = B.admit(torch.from_numpy(eta.reshape(q["cols"], -1)).cuda(), S_t, M=q["M"],
                                alpha=profile(DIMS[0], q["a0"], q["x0"]), r=r, x0_src=q["x0"], tag=k)
                q["S_t"] = S_t
                q["slots"] = slots
                return slots
            assert admit(0) is not None and admit(1) is not None
            assert admit(2) is None  # only 5 slots: the third request waits
            B.step(2)
            B.step(2)
            for res in B.harvest():
                got.setdefault(res["tag"], []).append(res)
            while B.status()["free"] < 1:
                B.step(2)
                for res in B.harvest():
                    got.setdefault(res["tag"], []).append(res)
            assert admit(2) is not None  # joins the running batch
            while B.status()["running"] or B.status()["done"]:
                B.step(3)
                for res in B.harvest():
                    got.setdefault(res["tag"], []).append(res)
        for k, q in enumerate(reqs):
            assert len(got[k]) == q["cols"]
            alpha = profile(DIMS[0], q["a0"], q["x0"])
            S_b = q["S_t"].cpu().numpy().reshape((q["cols"],) + DIMS + (4, 3))
            eta = point_columns(DIMS, q["x0"], q["cols"])
            cpp_b = {q["slots"].index(res["slot"]): res["cpp"] for res in got[k]}
            # solo solves of the same columns on a fresh context
            with lattice(DIMS) as L2:
                L2.set_gauge(U)
                L2.set_clover(1.6)
                for c in range(q["cols"]):
                    S1, cpp1, info1 = solo(L2, eta[c], q["M"], alpha, q["x0"], r, precision)
                    assert np.array_equal(S1, S_b[c]), (k, c)
                    assert np.array_equal(cpp1, cpp_b[c]), (k, c)
                    # stopping rule recomputed by the oracle
                    a6 = alpha[:, None, None, None, None, None]
                    res = a6 * eta[c] - oracle.apply(U, C, q["M"], a6 * S_b[c], alpha=alpha)
                    assert np.linalg.norm(res) <= 1.0001 * r * np.linalg.norm(a6 * eta[c])
            log(f"  request {k}: iters {[res['info']['iters'] for res in got[k]]}")


def test_server_poisson_stream_and_memory_gate():
    from paper_1006_4028_amd.serve import Server, poisson_requests, summarize, point_columns, profile
    log("test_server_poisson_stream_and_memory_gate")
    fields = {"a": ((8, 4, 4, 4), synth.gauge_su3((8, 4, 4, 4), 0.3, 1), 1.6),
              "b": ((6, 4, 4, 6), synth.gauge_su3((6, 4, 4, 6), 0.3, 2), 1.6)}
    reqs = poisson_requests(24, rate=400.0, fields=fields, T_of={"a": 8, "b": 6}, seed=3, max_cols=5)
    srv = Server(fields, nslots=8, precision="f32", r=1e-10)
    try:
        out = srv.run(reqs)
        s = summarize(srv, out)
    finally:
        srv.close()
    log("  ", s)
    assert s["done"] == 24 and s["failed"] == 0 and s["rejected"] == 0
    # every request equals the solo solve of its columns
    for q in out[:6]:
        dims, U, csw = fields[q.field]
        with lattice(dims) as L:
            L.set_gauge(U)
            L.set_clover(csw)
            L.set_mass(q.M)
            L.set_alpha(profile(dims[0], q.alpha0, q.x0))
            _, cpp, _ = L.solve(point_columns(dims, q.x0, q.ncols), r=1e-10, precision="f32", x0_src=q.x0,
                                ncols_group=q.ncols)
        assert np.allclose(q.cpp, cpp[0], rtol=1e-12, atol=0), q.rid
    # a budget that holds the fields and workspaces but only one inverse clover
    # per field rejects requests that need a second mass on the same field
    from paper_1006_4028_amd import footprint_bytes
    base = sum(footprint_bytes(d, 8, "f32", 0) for d, _, _ in fields.values())
    one = max(footprint_bytes(d, 0, "f32", 1) - footprint_bytes(d, 0, "f32", 0) for d, _, _ in fields.values())
    srv = Server(fields, nslots=8, precision="f32", r=1e-10, hbm_budget=base + 2 * one)
    try:
        out = srv.run(poisson_requests(16, rate=400.0, fields=fields, T_of={"a": 8, "b": 6}, seed=4, max_cols=3))
        s = summarize(srv, out)
    finally:
        srv.close()
    log("  gated:", s)
    assert s["rejected"] > 0 and s["done"] + s["rejected"] == 16


def test_batch_mass_change_after_shared_inverse():
    """A batch whose slots all hold one mass stages that mass's A_oo^-1 once
    per workgroup (FP32 multi-slot kernels), and its captured iteration graph
    bakes that in; requests of another mass admitted later must get their own
    inverse (the graph is captured again).  Every column equals its solo
    solve bit for bit."""
    import torch
    import paper_1006_4028_amd as dp
    from paper_1006_4028_amd.serve import point_columns, profile
    log("test_batch_mass_change_after_shared_inverse")
    U = synth.gauge_su3(DIMS, 0.4, 23)
    r = 1e-10
    reqs = [dict(M=0.5, a0=0.4, x0=0, cols=4), dict(M=0.05, a0=0.1, x0=2, cols=2),
            dict(M=0.5, a0=0.0, x0=5, cols=2)]
    with lattice(DIMS) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        got = {}
        with dp.Batch(L, 4, "f32") as B:
            def admit(k):
                q = reqs[k]
                eta = point_columns(DIMS, q["x0"], q["cols"])
                S_t = torch.zeros(q["cols"], eta[0].size, dtype=torch.complex128, device="cuda")
                slots = B.admit(torch.from_numpy(eta.reshape(q["cols"], -1)).cuda(), S_t, M=q["M"],
                                alpha=profile(DIMS[0], q["a0"], q["x0"]), r=r, x0_src=q["x0"], tag=k)
                q["S_t"] = S_t
                return slots

            def drain(until_free):
                while B.status()["free"] < until_free:
                    B.step(2)
                    for res in B.harvest():
                        got.setdefault(res["tag"], []).append(res)

            assert admit(0) is not None  # every slot at M = 0.5: shared inverse
            drain(4)
            assert admit(1) is not None  # M = 0.05 next to stale M = 0.5 slots
            assert admit(2) is not None  # and M = 0.5 again beside it
            drain(4)
        for k, q in enumerate(reqs):
            assert len(got[k]) == q["cols"]
            alpha = profile(DIMS[0], q["a0"], q["x0"])
            S_b = q["S_t"].cpu().numpy().reshape((q["cols"],) + DIMS + (4, 3))
            eta = point_columns(DIMS, q["x0"], q["cols"])
            with lattice(DIMS) as L2:
                L2.set_gauge(U)
                L2.set_clover(1.6)
                for c in range(q["cols"]):
                    S1, _, _ = solo(L2, eta[c], q["M"], alpha, q["x0"], r, "f32")
                    assert np.array_equal(S1, S_b[c]), (k, c)
            log(f"  request {k}: iters {[res['info']['iters'] for res in got[k]]}")
