"""The timeslice-range XCD mapping (DP_HOP_TMAP=1, read once per process):
a child process with the knob set applies the Schur operator to 1 and 12
right-hand sides and solves 12 columns; the operator results must equal the
default mapping's bitwise (the per-site arithmetic is the same, only the
blocks' order differs) and the solve's C_PP must agree within 1e-8 per
timeslice against each other (the reduction partition differs, so the dot
products round differently and the solves stop at different iterates of
the same residual).  The lattice has several chunks per XCD slab and a timeslice
count that does not divide by 8."""
import os
import subprocess
import sys

import numpy as np
import pytest

from gpu_common import log

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1]); sys.path.insert(0, sys.argv[1] + "/tests")
import paper_1006_4028_amd as dp, synth
dims = (12, 16, 12, 16)
U = synth.gauge_su3(dims, 0.5, 71)
L = dp.Lattice(dims)
L.set_gauge(U); L.set_clover(1.6); L.set_mass(0.4); L.set_alpha(synth.alpha_exp(dims[0], 0.3))
out = {}
for prec in ("f64", "f32", "f16"):
    for n in (1, 12):
        x = torch.from_numpy(synth.random_spinor(dims, 5, nrhs=n).reshape(n, -1)).cuda()
        y = torch.empty_like(x)
        L.apply_dev(x, y, precond=True, schur=True, precision=prec)
        out[f"{prec}_{n}"] = y.cpu().numpy()
eta = synth.point_sources_12(dims, (0, 0, 0, 0))
_, cpp, info = L.solve(eta, r=1e-11, precision="f32", ncols_group=12, want_S=False)
out["cpp"] = cpp
L.close()
np.savez(sys.argv[2], **out)
"""


def run_child(tmp_path, tmap):
    path = str(tmp_path / f"tmap{tmap}.npz")
    env = dict(os.environ, DP_HOP_TMAP=str(tmap))
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, path], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return np.load(path)


def test_time_mapping_matches_slab_mapping(tmp_path):
    log("test_time_mapping_matches_slab_mapping")
    a = run_child(tmp_path, 0)
    b = run_child(tmp_path, 1)
    for k in a.files:
        if k == "cpp":
            continue
        assert np.array_equal(a[k], b[k]), k
    err = np.abs(b["cpp"] / a["cpp"] - 1).max()
    log(f"  C_PP tmap vs slab max rel {err:.2e}")
    assert err < 1e-8
