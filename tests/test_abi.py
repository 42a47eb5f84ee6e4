"""The C-ABI library loads on the host and exports every entry point that
include/dp.h declares (no compute calls: there may be no GPU here)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|long long|const char\s*\*)\s+(dp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dp_create", "dp_set_gauge", "dp_set_clover", "dp_set_mass", "dp_set_alpha", "dp_apply",
              "dp_solve", "dp_solve_dev", "dp_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1006_4028_amd as dp
    L = dp._lib.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", dp._lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (dp_\w+)", out))
    assert set(declared_functions()) <= exported
    assert set(dp._lib.EXPORTED) == set(declared_functions())


def test_footprint_is_host_only_and_validates():
    import paper_1006_4028_amd as dp
    a = dp.footprint_bytes((48, 24, 24, 24), 1, "f32")
    b = dp.footprint_bytes((48, 24, 24, 24), 12, "f32")
    c = dp.footprint_bytes((48, 24, 24, 24), 12, "f64")
    assert 0 < a < b < c
    assert dp.footprint_bytes((48, 24, 23, 24), 1, "f32") == -1


def test_binding_has_no_fallback(tmp_path, monkeypatch):
    """Without libdp.so the binding raises instead of computing elsewhere."""
    import paper_1006_4028_amd._lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.lib()


def test_hop_kernels_do_not_spill():
    """The compiler's resource report of the last build: no hop kernel
    instantiation spills registers to scratch memory (a spill made the FP64
    even-site kernel twice as slow once; the build records the report)."""
    import json
    path = os.path.join(ROOT, "paper_1006_4028_amd", "_build", "kernel_resources.json")
    if not os.path.exists(path):
        pytest.skip("no build report (run paper_1006_4028_amd/build.py)")
    res = json.load(open(path))
    hops = {k: v for k, v in res.items() if "hop_kernel" in k}
    assert hops
    spill = {k: v for k, v in hops.items() if v.get("scratch", 0) > 0}
    assert not spill, spill
