"""dp_apply_dev_noalloc (the entry point for callers that cannot allocate
device memory) against dp_apply_dev through the C ABI: the same flags and
inputs give bitwise the same output, on two calls in a row, the second with
fewer right-hand sides, in every precision; the device's free memory does
not change across the calls; requests beyond the static scratch, and a Schur
operator whose inverse clover was never built, are refused with an error
(host-side checks, before any launch)."""
import numpy as np
import pytest

import synth
from gpu_common import lattice, log

pytestmark = pytest.mark.gpu


def test_noalloc_matches_apply_dev_two_calls():
    import torch
    import paper_1006_4028_amd as dp
    dims = (8, 4, 6, 4)
    log("test_noalloc_matches_apply_dev_two_calls")
    U = synth.gauge_su3(dims, 0.3, 71)
    alpha = synth.alpha_exp(dims[0], 0.3)
    psi = synth.random_spinor(dims, 72, nrhs=5)
    with lattice(dims) as L:
        L.set_gauge(U)
        L.set_clover(1.6)
        L.set_mass(0.2)
        L.set_alpha(alpha)
        x = torch.from_numpy(psi.reshape(5, -1)).cuda()
        ref = torch.empty_like(x)
        # refused before anything runs: the inverse clover of M = 0.2 is not built yet
        with pytest.raises(dp.DPError) as e:
            L.apply_dev_noalloc(x, torch.empty_like(x), precond=True, schur=True)
        assert e.value.code == -7
        L.apply_dev(x, ref, precond=True, schur=True)  # builds it
        torch.cuda.synchronize()
        for precision in ("f64", "f32", "f16"):
            for flags in (dict(schur=True), dict(schur=True, dagger=True), dict(), dict(hop_only=True)):
                for n in (5, 2):  # the second call is smaller
                    xs = x[:n].contiguous()
                    want = torch.empty_like(xs)
                    got = torch.full_like(xs, float("nan"))
                    L.apply_dev(xs, want, precond=True, precision=precision, **flags)
                    torch.cuda.synchronize()
                    free0 = torch.cuda.mem_get_info()[0]
                    L.apply_dev_noalloc(xs, got, precond=True, precision=precision, **flags)
                    torch.cuda.synchronize()
                    free1 = torch.cuda.mem_get_info()[0]
                    assert free1 == free0, (precision, flags, n, free0 - free1)
                    assert torch.equal(got, want), (precision, flags, n)
        log("  bitwise equal to dp_apply_dev in f64/f32/f16, 5 then 2 right-hand sides")


def test_noalloc_rejects_too_large():
    import ctypes
    import torch
    import paper_1006_4028_amd as dp
    dims = (32, 16, 16, 16)  # one FP32 right-hand side needs 82 MB of the 128 MiB: two do not fit
    log("test_noalloc_rejects_too_large")
    with lattice(dims) as L:
        L.set_mass(0.5)
        x = torch.zeros((2, L.V * 12), dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        L.apply_dev_noalloc(x[:1], y[:1], precision="f32")  # fits
        with pytest.raises(dp.DPError) as e:
            L.apply_dev_noalloc(x, y, precision="f32")
        assert e.value.code == -1 and "scratch" in L._L.dp_last_error(L._h).decode()
        # more right-hand sides than DP_NOALLOC_MAX_RHS: refused before any pointer is used
        rc = L._L.dp_apply_dev_noalloc(L._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       dp._lib.DP_NOALLOC_MAX_RHS + 1, 0, None)
        assert rc == -1
