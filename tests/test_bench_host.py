"""Host logic of bench.py (no GPU): the one-GPU guard, the counter summary
(FETCH_SIZE / WRITE_SIZE scaled by what they read for a copy of known size)
and the rule that a counter record only counts for the kernel sources it was
taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def _csv(path, rows):
    with open(path, "w") as f:
        f.write('"Kernel_Name","Counter_Value"\n')
        for name, v in rows:
            f.write(f'"{name}",{v}\n')


def test_counter_summary_scales_by_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    hop = "void dp::(anonymous namespace)::hop_kernel_shared<1, 2, 1, 1, true, false, false>(dp::HopArgs, x)"
    hop4 = "void dp::(anonymous namespace)::hop_kernel_shared<1, 2, 4, 1, true, false, false>(dp::HopArgs, x)"
    inv = "void dp::(anonymous namespace)::hop_kernel_shared<1, 1, 0, 1, true, false, true>(dp::HopArgs, x)"
    h16 = "void dp::(anonymous namespace)::hop_kernel_slab<2, 2, 4, 1, true, false>(dp::HopArgs, x)"
    # the 1 GiB copy reads as half its size in FETCH_SIZE and exactly in WRITE_SIZE;
    # a launch with few active slots (the last hop one) is left out of the mean
    _csv(tmp_path / "f.csv", [("__amd_rocclr_copyBuffer", 524288), (hop, 1000.0), (hop4, 1200.0), (hop, 100.0),
                              (inv, 5000.0), (h16, 700.0)])
    _csv(tmp_path / "w.csv", [("__amd_rocclr_copyBuffer", 1048576), (hop, 300.0), (hop4, 300.0), (hop, 30.0),
                              (inv, 900.0), (h16, 200.0)])
    (tmp_path / "alg.json").write_text(json.dumps({"alg_bytes_per_launch": {"hop_f32_diag": 1024 * 2000.0}}))
    bench.pmc_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "alg.json"), "cmd")
    rec = json.load(open(tmp_path / "traffic.json"))
    assert rec["fetch_scale"]["scale"] == 2.0 and rec["write_scale"]["scale"] == 1.0
    k = rec["kernels"]
    assert set(k) == {"hop_f32_diag", "hop_f32_inv", "hop_f16_diag"}
    assert k["hop_f32_diag"]["launches"] == 2
    assert k["hop_f32_diag"]["hbm_bytes_per_launch"] == 1024 * (1100.0 * 2.0 + 300.0)
    assert k["hop_f32_diag"]["traffic_over_alg"] == round((1100.0 * 2.0 + 300.0) / 2000.0, 3)
    assert k["hop_f32_inv"]["hbm_bytes_per_launch"] == 1024 * (5000.0 * 2.0 + 900.0)
    assert k["hop_f32_inv"]["traffic_over_alg"] is None
    assert k["hop_f16_diag"]["hbm_bytes_per_launch"] == 1024 * (700.0 * 2.0 + 200.0)
    assert rec["source_sha256"] == bench.kernel_source_hash()


def test_counter_record_of_other_sources_is_ignored(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    rec = {"kernels": {"hop_f32_diag": {"hbm_bytes_per_launch": 2.5}}}
    json.dump({"source_sha256": "0" * 64, **rec}, open(path, "w"))
    assert bench.measured_traffic() is None
    json.dump({"source_sha256": bench.kernel_source_hash(), **rec}, open(path, "w"))
    assert bench.measured_traffic() == 2.5
    assert bench.measured_traffic("hop_f16_inv") is None
