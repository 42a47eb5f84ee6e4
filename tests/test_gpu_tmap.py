"""The two XCD mappings (spatial slabs and timeslice ranges, forced with
DP_HOP_TMAP = 0 / 1, read once per process): a child process per mapping
applies the Schur operator to 1 and 12 right-hand sides and solves 12
columns; everything must be bitwise the same (the per-site arithmetic and
the reduction partition, one partial per timeslice and chunk, do not depend
on the mapping; only the blocks' order differs).  The lattice has several
chunks per XCD slab and a timeslice count that does not divide by 8."""
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
        assert np.array_equal(a[k], b[k]), k
