#!/usr/bin/env python3
"""Benchmark of the distance-preconditioned Wilson-clover solve on one MI355X.

One step = one 12-column point-source propagator of the 24^3 x 48 workload
(synthetic SU(3) field, eps = 0.25, c_sw = 1.6, M = 0.5, the paper's
periodic-time profile with alpha0 = 0.4, r = 1e-11): source redefinition,
Schur right-hand side, the mixed-precision solve (FP32 inner BiCGStab, FP64
residuals and updates), odd-site reconstruction, restoration S = S'/alpha
and C_PP, with eta and S resident in HBM.  `value` counts solved
right-hand sides per second.  The same steps on the FP64 path, the per-
timeslice C_PP agreement of the two, the dominant kernel's roofline (from
HIP events on the library's stream) and the CPU oracle on one column are
reported on the same line.

The timed steps run the production path: each batch of inner iterations is
replayed from a captured hipGraph and no launch is bracketed by events.  The
per-kernel roofline comes from a separate pass of two steps with HIP events
around every launch on the library's stream (graphs off).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash HBM GB/s (% roofline); solves/s + p99 latency, mixed vs FP64 at r=1e-11"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_hop_kernels_24c48_12rhs.json")
KERNEL_SOURCES = ["paper_1006_4028_amd/csrc/hop.hip", "paper_1006_4028_amd/csrc/dp_device.h",
                  "paper_1006_4028_amd/csrc/dp_common.h"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel="hop_f32_diag"):
    """HBM bytes per full launch of a hop kernel class from the committed
    counter record, if it was taken on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["hbm_bytes_per_launch"]


def pmc_probe():
    """Run under rocprofv3 --pmc: a 1 GiB device copy (the counters' scale),
    then one solve of the timed configuration (12 columns) with FP32 and one
    with FP16 inner precision, with per-kernel timing on (graphs off), and
    print the algorithmic bytes per launch of each hop kernel class as one
    JSON line."""
    import torch
    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    import paper_1006_4028_amd as dp
    import synth
    cfg = synth.config("su3_24c48")
    dims = cfg["dims"]
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), 12)
    e_t = torch.from_numpy(eta.reshape(12, -1)).cuda()
    L = dp.Lattice(dims)
    L.set_gauge(U)
    L.set_clover(cfg["csw"])
    L.set_mass(cfg["masses"][0])
    L.set_alpha(synth.alpha_table(cfg["profile"], dims[0], cfg["alpha0s"][-1]))
    alg = {}
    for prec in ("f32", "f16"):
        L.set_timing(True)
        L.solve_dev(e_t, None, r=cfg["r"], precision=prec, ncols_group=12)
        torch.cuda.synchronize()
        for name, st in L.timing().items():
            if name.startswith("hop_") and st["launches"]:
                alg[name] = max(alg.get(name, 0.0), st["bytes"] / st["launches"])
        L.set_timing(False)
    L.close()
    print(json.dumps({"alg_bytes_per_launch": alg}), flush=True)


# counter-record kernel classes: (timer name, test on the kernel's template
# arguments <precision, epilogue, ...>)
PMC_CLASSES = {
    "hop_f32_diag": lambda a: a[0] == 1 and a[1] == 2,
    "hop_f32_inv": lambda a: a[0] == 1 and a[1] in (1, 4),
    "hop_f16_diag": lambda a: a[0] == 2 and a[1] == 2,
    "hop_f16_inv": lambda a: a[0] == 2 and a[1] in (1, 4),
}


def pmc_summary(fetch_csv, write_csv, alg_json, command):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the 12-slot hop
    kernels by what the same counters read for the 1 GiB copy, average them
    over the full launches of each kernel class (every slot active) and
    record them with the algorithmic bytes of the same launches."""
    import csv
    import re

    def rows(path):
        return list(csv.DictReader(open(path)))

    def is_copy(r):
        return "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"].lower() and "dp::" not in r["Kernel_Name"]

    def targs(r):
        m = re.search(r"hop_kernel_(?:shared|slab)<([^>]*)>", r["Kernel_Name"])
        return None if not m else [int(v) if v.strip().lstrip("-").isdigit() else v.strip() for v in m.group(1).split(",")]

    line = [x for x in open(alg_json).read().splitlines() if '"alg_bytes_per_launch"' in x][-1]
    alg = json.loads(line)["alg_bytes_per_launch"]
    scale, per = {}, {}
    for key, path in (("fetch", fetch_csv), ("write", write_csv)):
        rs = rows(path)
        copy = max(float(r["Counter_Value"]) for r in rs if is_copy(r))
        scale[key] = {"copy_kib": copy, "scale": (1 << 20) / copy}  # the copy moves 1 GiB = 2^20 KiB
        for cls, test in PMC_CLASSES.items():
            vals = [float(r["Counter_Value"]) for r in rs if targs(r) and test(targs(r))]
            if not vals:
                continue
            full = [v for v in vals if v > 0.5 * max(vals)]
            per.setdefault(cls, {})[key] = (sum(full) / len(full), len(full))
    kernels = {}
    for cls, d in per.items():
        if "fetch" not in d or "write" not in d:
            continue
        hbm = 1024 * (d["fetch"][0] * scale["fetch"]["scale"] + d["write"][0] * scale["write"]["scale"])
        a = alg.get(cls)
        kernels[cls] = {"hbm_bytes_per_launch": hbm, "fetch_kib_per_launch": d["fetch"][0],
                        "write_kib_per_launch": d["write"][0], "launches": d["fetch"][1],
                        "alg_bytes_per_launch": a, "traffic_over_alg": None if not a else round(hbm / a, 3)}
    rec = {"workload": "24^3x48, 12 slots, one FP32-inner and one FP16-inner solve to r=1e-11",
           "command": command, "source_sha256": kernel_source_hash(),
           "fetch_scale": scale["fetch"], "write_scale": scale["write"], "kernels": kernels}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# C_PP of the 12 point-source columns from the FP64 oracle (written by
# tests/golden/make_golden.py, which calls only oracle/)
GOLDEN = {"su3_16c32": "tests/golden/cpp_su3_16c32_M0.5.txt", "su3_24c48": "tests/golden/cpp_su3_24c48_M0.5.txt"}


def load_golden(workload):
    import numpy as np
    path = GOLDEN.get(workload)
    if path is None or not os.path.exists(os.path.join(ROOT, path)):
        return None
    return np.loadtxt(os.path.join(ROOT, path))[:, 1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="su3_24c48")
    ap.add_argument("--precision", default="f32", choices=["f32", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests in the served stream at the arrival rate (0 skips the serving measurement)")
    ap.add_argument("--serve-capacity-requests", type=int, default=120,
                    help="requests submitted at once to measure the capacity")
    ap.add_argument("--serve-rate", type=float, default=5.0,
                    help="Poisson arrival rate of the stream, 1/s (5/s is about 0.8 of the FP64-inner capacity)")
    ap.add_argument("--serve-r", type=float, default=1e-11, help="residue of the served requests")
    ap.add_argument("--roofline-steps", type=int, default=2, help="event-timed steps for the per-kernel roofline")
    ap.add_argument("--no-dslash", action="store_true", help="skip the operator (Dslash) benchmark")
    ap.add_argument("--dslash-calls", type=int, default=200, help="timed operator calls per case")
    ap.add_argument("--sap-study", action="store_true",
                    help="SAP+GCR iteration counts vs alpha0 of the light-quark factorisation (one JSON line)")
    ap.add_argument("--sap-workload", default=None, choices=["su3_24c48", "su3_32c64"],
                    help="with --sap-study: only this lattice")
    ap.add_argument("--pmc-probe", action="store_true", help="run the counter probe (under rocprofv3 --pmc)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "ALG_JSON", "COMMAND"),
                    help="write the traffic record of the dominant kernel from two counter runs")
    args = ap.parse_args()
    if args.pmc_probe:
        return pmc_probe()
    if args.pmc_summary:
        return pmc_summary(*args.pmc_summary)
    if args.sap_study:
        return sap_study(args.sap_workload, not args.no_cpu_baseline)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one process drives one GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1006_4028_amd as dp
    import synth

    cfg = synth.config(args.workload)
    dims, M, csw, r = cfg["dims"], cfg["masses"][0], cfg["csw"], cfg["r"]
    alpha0 = cfg["alpha0s"][-1]
    ncols = 12
    log(f"workload {args.workload} dims={dims}: generating the field")
    U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
    alpha = synth.alpha_table(cfg["profile"], dims[0], alpha0)
    eta = synth.point_sources_12(dims, (0, 0, 0, 0), ncols)

    dev = torch.device("cuda:0")
    eta_t = torch.from_numpy(eta.reshape(ncols, -1)).to(dev)
    S_t = torch.empty_like(eta_t)
    L = dp.Lattice(dims)
    L.set_gauge(U)
    L.set_clover(csw)
    L.set_mass(M)
    L.set_alpha(alpha)

    def run(precision, steps, warmup, timing=False):
        for _ in range(warmup):
            L.solve_dev(eta_t, S_t, r=r, precision=precision, ncols_group=ncols)
        L.set_timing(timing)
        lat, infos, cpp = [], None, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            cpp, infos = L.solve_dev(eta_t, S_t, r=r, precision=precision, ncols_group=ncols)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        stats = L.timing() if timing else {}
        L.set_timing(False)
        return total, lat, infos, cpp, stats

    log(f"mixed path ({args.precision} inner): {args.warmup} warmup + {args.steps} timed steps (graph replay)")
    total, lat, infos, cpp_mixed, _ = run(args.precision, args.steps, args.warmup)
    for i in infos:
        assert i["status"] == 0 and i["true_res"] <= r, i
    solves_per_s = ncols * args.steps / total
    lat_ms = sorted(1e3 * x for x in lat)
    log(f"roofline pass: {args.roofline_steps} steps with HIP events around every launch (graphs off)")
    t_ev, _, _, _, stats = run(args.precision, args.roofline_steps, 0, timing=True)
    golden = load_golden(args.workload)

    def vs_oracle(cpp):
        return None if golden is None else float(np.abs(cpp / golden - 1).max())

    def pct(v, q):
        k = min(len(v) - 1, max(0, int(round(q * (len(v) - 1)))))
        return v[k]

    # dominant kernel: the hop variant with the most total time
    hops = {k: v for k, v in stats.items() if k.startswith("hop_")}
    name, st = max(hops.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = st["ms"] / st["launches"]
    gbs = st["bytes"] / st["launches"] / (avg_ms * 1e-3) / 1e9
    # a measured streaming rate of this library: s = r - alpha v (two vectors
    # read, one written, no neighbours)
    stream = stats.get(f"blas_{args.precision}_4")
    stream_gbs = stream["bytes"] / (stream["ms"] * 1e-3) / 1e9 if stream and stream["ms"] > 0 else None
    all_hop_ms = sum(v["ms"] for v in hops.values())
    all_hop_gbs = sum(v["bytes"] for v in hops.values()) / (all_hop_ms * 1e-3) / 1e9
    log(f"  {solves_per_s:.1f} solves/s, p50 {pct(lat_ms, 0.5):.2f} ms, p99 {pct(lat_ms, 0.99):.2f} ms, "
        f"iters {[i['iters'] for i in infos]}; event-timed pass {1e3 * t_ev / args.roofline_steps:.1f} ms per step")
    if golden is not None:
        log(f"  C_PP vs the FP64 oracle (stored correlator), max per-timeslice rel err {vs_oracle(cpp_mixed[0]):.2e}")
    for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["ms"]):
        log(f"  {k:18s} launches {v['launches']:6d} avg {1e3 * v['ms'] / v['launches']:8.1f} us "
            f"{v['bytes'] / (v['ms'] * 1e-3) / 1e9 if v['ms'] > 0 else 0:8.1f} GB/s")

    fp64 = None
    if not args.no_fp64:
        log(f"FP64 path: 1 warmup + {args.steps} timed steps")
        t64, lat64, infos64, cpp64, _ = run("f64", args.steps, 1)
        for i in infos64:
            assert i["status"] == 0 and i["true_res"] <= r, i
        lat64_ms = sorted(1e3 * x for x in lat64)
        cpp_err = float(np.abs(cpp_mixed[0] / cpp64[0] - 1).max())
        fp64 = {"value": round(ncols * args.steps / t64, 3), "unit": "solves/s",
                "p50_ms": round(pct(lat64_ms, 0.5), 3), "p99_ms": round(pct(lat64_ms, 0.99), 3),
                "iters": [i["iters"] for i in infos64],
                "mixed_vs_fp64_cpp_max_rel_err_per_timeslice": cpp_err,
                "cpp_vs_oracle_max_rel_err_per_timeslice": vs_oracle(cpp64[0])}
        log(f"  {fp64['value']} solves/s; mixed/FP64 C_PP max rel err per timeslice {cpp_err:.2e}")
        if args.precision == "f32":
            # the lowest rung of the precision ladder, FP16 storage with per-site scales
            log(f"FP16-storage inner path: 1 warmup + {args.steps} timed steps")
            t16, lat16, infos16, cpp16, _ = run("f16", args.steps, 1)
            for i in infos16:
                assert i["status"] == 0 and i["true_res"] <= r, i
            lat16_ms = sorted(1e3 * x for x in lat16)
            fp64["f16_inner"] = {"value": round(ncols * args.steps / t16, 3), "unit": "solves/s",
                                 "p50_ms": round(pct(lat16_ms, 0.5), 3), "p99_ms": round(pct(lat16_ms, 0.99), 3),
                                 "iters": [i["iters"] for i in infos16],
                                 "vs_fp64_cpp_max_rel_err_per_timeslice":
                                     float(np.abs(cpp16[0] / cpp64[0] - 1).max()),
                                 "cpp_vs_oracle_max_rel_err_per_timeslice": vs_oracle(cpp16[0])}
            log(f"  {fp64['f16_inner']}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("CPU oracle: one column of the same workload, FP64 BiCGStab to r")
        C = oracle.clover(U, csw)
        t0 = time.perf_counter()
        _, info_or = oracle.solve(U, C, M, eta[0], alpha=alpha, r=r)
        t_or = time.perf_counter() - t0
        cpu = {"value": round(1.0 / t_or, 6), "unit": "solves/s", "cores": oracle.get_threads(), "kind": "oracle",
               "sample": f"1 of the {ncols} columns, full-lattice FP64 BiCGStab, {info_or['iters']} iterations, "
                         f"{t_or:.1f} s"}
        log(f"  {t_or:.1f} s for one column on {cpu['cores']} threads")
        # the oracle's full-lattice operator on all threads and on one: links
        # 144 + clover 72 + input 24 + output 24 reals per site, FP64
        V = int(np.prod(dims))
        nthr = oracle.get_threads()
        cpu["operator"] = []
        for n in (nthr, 1):
            oracle.set_threads(n)
            oracle.apply(U, C, M, eta[0], alpha=alpha)
            t0 = time.perf_counter()
            for _ in range(3):
                oracle.apply(U, C, M, eta[0], alpha=alpha)
            t_ap = (time.perf_counter() - t0) / 3
            cpu["operator"].append({"threads": n, "ms": round(1e3 * t_ap, 1),
                                    "GBps": round(V * 264 * 8 / t_ap / 1e9, 2)})
            log(f"  oracle operator on {n} threads: {1e3 * t_ap:.1f} ms")
        oracle.set_threads(nthr)
        cpu["configs"] = oracle_config_timings(oracle, nthr)

    traffic = measured_traffic()
    L.close()
    dslash = None if args.no_dslash else dslash_bench(args)
    serving = None
    if args.serve_requests > 0:
        serving = serve_stream(args, cfg)

    out = {
        "metric": METRIC,
        "value": round(solves_per_s, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 outer" if args.precision == "f32" else "f16 storage inner / f64 outer",
        "data": "synthetic (seeded SU(3) field, point sources)",
        "config": {"workload": f"{args.workload}: {dims[1]}^3x{dims[0]} clover c_sw={csw}, M={M}, "
                               f"{cfg['profile']} alpha0={alpha0}, {ncols} point-source columns per step, r={r}",
                   "global_batch": ncols, "parallelism": "single GPU"},
        "p50_ms": round(pct(lat_ms, 0.5), 3),
        "p99_ms": round(pct(lat_ms, 0.99), 3),
        "iters": [i["iters"] for i in infos],
        "cpp_vs_oracle_max_rel_err_per_timeslice": vs_oracle(cpp_mixed[0]),
        "cpp_oracle_reference": None if golden is None else GOLDEN[args.workload],
        "event_timed_ms_per_step": round(1e3 * t_ev / args.roofline_steps, 3),
        "fp64": fp64,
        "speedup_vs_fp64": round(solves_per_s / fp64["value"], 3) if fp64 else None,
        "roofline": {"bound": "hbm", "kernel": name, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_over_alg": round(traffic / (st["bytes"] / st["launches"]), 3) if traffic else None,
                     "avg_launch_us": round(1e3 * avg_ms, 2),
                     "alg_bytes_per_launch": st["bytes"] / st["launches"],
                     "all_hop_kernels_GBps": round(all_hop_gbs, 1),
                     "stream_GBps": round(stream_gbs, 1) if stream_gbs else None,
                     "frac_of_stream": round(gbs / stream_gbs, 4) if stream_gbs else None},
        "cpu_baseline": cpu,
        "dslash": dslash,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


def sap_study(only=None, cpu_baseline=True):
    """The analogue of the paper's Table 1 on the synthetic fields: SAP+GCR
    iterations (and seconds) to invert the light-quark Dirac equation with the
    four-direction cosh factorisation (eq. betaa) for alpha0 in {0, 0.2, 0.4};
    48 x 24^3 with 6^4 blocks at r = 1e-11 (the D5 shape) and 64 x 32^3 with
    4^4 blocks at r = 1e-10 (the E shape); M in {0.01, 0.05}; FP32 block
    solves, ncy = 5, nmr = 4, nkv = 16; one point-source column, source and
    solution resident on the device (the seconds exclude host transfers).
    The CPU baseline leg times one application of the oracle's SAP
    preconditioner (M = 0.05, alpha0 = 0.4) on each lattice, against the
    GPU's time per GCR iteration (one application, the FP64 operator and the
    Gram-Schmidt step)."""
    import numpy as np
    import torch
    import paper_1006_4028_amd as dp
    import synth
    out, cpu = [], []
    for name, block, r in (("su3_24c48", (6, 6, 6, 6), 1e-11), ("su3_32c64", (4, 4, 4, 4), 1e-10)):
        if only and name != only:
            continue
        cfg = synth.config(name)
        dims = cfg["dims"]
        U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
        L = dp.Lattice(dims)
        L.set_gauge(U)
        del U
        L.set_clover(cfg["csw"])
        eta = synth.point_sources_12(dims, (0, 0, 0, 0))[0]
        eta_t = torch.from_numpy(np.ascontiguousarray(eta)).cuda()
        S_t = torch.zeros_like(eta_t)
        for M in (0.01, 0.05):
            L.set_mass(M)
            for a0 in (0.0, 0.2, 0.4):
                L.set_beta(synth.beta_cosh_paper(dims, a0))
                _, info = L.solve_sap_dev(eta_t, S_t, block, r=r, max_iter=2000)
                rec = {"workload": name, "block": block, "r": r, "M": M, "alpha0": a0, "iters": info["iters"],
                       "restarts": info["outer"], "seconds": round(info["seconds"], 3),
                       "true_res": info["true_res"], "status": info["status"]}
                log(json.dumps(rec))
                out.append(rec)
        L.close()
        del eta_t, S_t
        if cpu_baseline:
            import oracle
            U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
            C = oracle.clover(U, cfg["csw"])
            r_h = synth.random_spinor(dims, 51)
            log(f"CPU oracle: one SAP application on {name}")
            t0 = time.perf_counter()
            oracle.sap_apply(U, C, 0.05, r_h, block, beta=synth.beta_cosh_paper(dims, 0.4))
            t_or = time.perf_counter() - t0
            del U, C, r_h
            per_it = min(x["seconds"] / x["iters"] for x in out if x["workload"] == name)
            rec = {"workload": name, "kind": "oracle", "cores": oracle.get_threads(),
                   "oracle_sap_apply_s": round(t_or, 2), "gpu_ms_per_gcr_iteration": round(1e3 * per_it, 2)}
            log(json.dumps(rec))
            cpu.append(rec)
    print(json.dumps({"sap_study": out, "cpu_baseline": cpu}), flush=True)


MALL_BYTES = 256 * 2 ** 20


def oracle_config_timings(oracle, nthr):
    """The oracle on the other workloads, all threads: one FP64 BiCGStab column
    to r = 1e-11 on the free 8^3x16 and the 16^3x32 fields, and the
    full-lattice operator (GB/s as for the main workload) on those and on
    32^3x64 (its light-mass solve is left out: hundreds of iterations)."""
    import numpy as np
    import synth
    out = []
    for name in ("free_8c16", "su3_16c32", "su3_32c64"):
        cfg = synth.config(name)
        dims = cfg["dims"]
        U = synth.free_gauge(dims) if cfg["eps"] == 0 else synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
        C = None if cfg["csw"] == 0 else oracle.clover(U, cfg["csw"])
        M = cfg["masses"][0]
        alpha = synth.alpha_table(cfg["profile"], dims[0], cfg["alpha0s"][-1])
        eta = synth.point_sources_12(dims, (0, 0, 0, 0), 1)[0]
        V = int(np.prod(dims))
        rec = {"workload": name, "threads": nthr}
        oracle.apply(U, C, M, eta, alpha=alpha)
        t0 = time.perf_counter()
        for _ in range(3):
            oracle.apply(U, C, M, eta, alpha=alpha)
        t_ap = (time.perf_counter() - t0) / 3
        rec["operator_ms"] = round(1e3 * t_ap, 2)
        rec["operator_GBps"] = round(V * 264 * 8 / t_ap / 1e9, 2)
        if name != "su3_32c64":
            t0 = time.perf_counter()
            _, info = oracle.solve(U, C, M, eta, alpha=alpha, r=1e-11)
            rec["solve_s"] = round(time.perf_counter() - t0, 3)
            rec["solve_iters"] = info["iters"]
        out.append(rec)
        log(f"  oracle {name}: {rec}")
    return out


def dslash_bench(args):
    """The even-site Schur operator (hop with A_oo^-1 on odd sites, then hop
    with the clover diagonal on even sites) of the preconditioned system on
    device-resident spinors, 24^3x48 (M = 0.5, cosh alpha0 = 0.4) and 32^3x64
    (M = 0.01, symmetric exp alpha0 = 0.1), in FP64, FP32 and FP16 storage,
    with 1 and 12 right-hand sides: 20 untimed calls, then per-launch HIP-event
    durations of each hop kernel over the timed calls (median, p10, p90) and
    the algorithmic HBM rate at the median.  Launches whose algorithmic bytes
    fit the 256 MB MALL are flagged."""
    import numpy as np
    import torch

    import paper_1006_4028_amd as dp
    import synth

    # a measured streaming rate beside the 8 TB/s specification: a 2 GiB
    # device-to-device copy (read + write)
    a = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ts = []
    for _ in range(20):
        ev[0].record()
        b.copy_(a)
        ev[1].record()
        ev[1].synchronize()
        ts.append(ev[0].elapsed_time(ev[1]) * 1e-3)
    copy_gbs = 2 * a.numel() * 4 / float(np.median(ts)) / 1e9
    del a, b
    log(f"operator benchmark: device copy {copy_gbs:.0f} GB/s")
    out = []
    for name, a0 in (("su3_24c48", 0.4), ("su3_32c64", 0.1)):
        cfg = synth.config(name)
        dims = cfg["dims"]
        log(f"operator benchmark {name}: {args.dslash_calls} timed calls per case")
        U = synth.gauge_su3(dims, cfg["eps"], cfg["seed"])
        L = dp.Lattice(dims)
        L.set_gauge(U)
        del U
        L.set_clover(cfg["csw"])
        L.set_mass(cfg["masses"][0])
        L.set_alpha(synth.alpha_table(cfg["profile"], dims[0], a0))
        V = int(np.prod(dims))
        for nrhs in (1, 12):
            gen = torch.Generator(device="cuda").manual_seed(nrhs)
            x = torch.randn(nrhs, V * 12, dtype=torch.complex128, device="cuda", generator=gen)
            y = torch.empty_like(x)
            for prec in ("f64", "f32", "f16"):
                for _ in range(20):
                    L.apply_dev(x, y, precond=True, schur=True, precision=prec)
                L.set_timing(True)
                for _ in range(args.dslash_calls):
                    L.apply_dev(x, y, precond=True, schur=True, precision=prec)
                st = L.timing()
                for k in sorted(st):
                    if not k.startswith("hop_"):
                        continue
                    us = 1e3 * L.timing_samples(k)
                    med = float(np.median(us))
                    b = st[k]["bytes"] / st[k]["launches"]
                    rec = {"workload": name, "precision": prec, "nrhs": nrhs, "kernel": k,
                           "launches": st[k]["launches"], "median_us": round(med, 2),
                           "p10_us": round(float(np.percentile(us, 10)), 2),
                           "p90_us": round(float(np.percentile(us, 90)), 2),
                           "alg_bytes": b, "GBps": round(b / (med * 1e-6) / 1e9, 1),
                           "frac": round(b / (med * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                           "copy_GBps": round(copy_gbs, 1),
                           "frac_of_copy": round(b / (med * 1e-6) / 1e9 / copy_gbs, 4),
                           "mall_resident": b < MALL_BYTES}
                    out.append(rec)
                    log(f"  {prec} nrhs={nrhs:2d} {k:14s} median {med:8.1f} us  {rec['GBps']:7.1f} GB/s "
                        f"({100 * rec['frac']:.1f}%){'  MALL-resident' if rec['mall_resident'] else ''}")
                L.set_timing(False)
            del x, y
        L.close()
    return out


def serve_stream(args, cfg3):
    """The served stream: resident 16^3x32 and 24^3x48 fields, each request
    drawing M from {0.01, 0.05, 0.2, 0.5}, alpha0 from {0, 0.1, 0.4} and 1-12
    point-source columns at a random x0; batched solves to the residue of the
    metric (r = 1e-11 by default) with the FP32 inner solver and with the FP64
    one.  Each is run twice: a stream of requests all arriving at once (the
    capacity, solves/s) and Poisson arrivals at the given rate (latency,
    p50/p99 over --serve-requests requests)."""
    import synth
    from paper_1006_4028_amd.serve import Server, poisson_requests, summarize
    cfg2 = synth.config("su3_16c32")
    fields = {"16c32": (cfg2["dims"], synth.gauge_su3(cfg2["dims"], cfg2["eps"], cfg2["seed"]), cfg2["csw"]),
              "24c48": (cfg3["dims"], synth.gauge_su3(cfg3["dims"], cfg3["eps"], cfg3["seed"]), cfg3["csw"])}
    T_of = {k: v[0][0] for k, v in fields.items()}
    out = {"workload": "16^3x32 + 24^3x48 resident, M in {0.01,0.05,0.2,0.5}, alpha0 in {0,0.1,0.4} "
                       f"(exp of min(t,T-t)), 1-12 columns at random x0, r={args.serve_r}, 24 slots per field",
           "r": args.serve_r, "rate_per_s": args.serve_rate, "requests": args.serve_requests,
           "capacity_requests": args.serve_capacity_requests}

    def run(prec, rate, n):
        reqs = poisson_requests(n, rate, fields, T_of, seed=2024)
        srv = Server(fields, nslots=24, precision=prec, r=args.serve_r, max_iter=20000, k=4)
        try:
            s = summarize(srv, srv.run(reqs))
        finally:
            srv.close()
        log(f"  {s}")
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()}

    for prec in ("f32", "f64"):
        log(f"served stream, {prec} inner, r={args.serve_r}: {args.serve_capacity_requests} requests at once, "
            f"then {args.serve_requests} at {args.serve_rate}/s")
        cap = run(prec, 1e6, args.serve_capacity_requests)
        lat = run(prec, args.serve_rate, args.serve_requests)
        out[prec] = {"capacity_solves_per_s": cap["solves_per_s"], "capacity_run": cap, "at_rate": lat}
    if out["f64"]["capacity_solves_per_s"] > 0:
        out["mixed_over_fp64_capacity"] = round(out["f32"]["capacity_solves_per_s"] /
                                                out["f64"]["capacity_solves_per_s"], 3)
    if out["f32"]["at_rate"]["p50_ms"] > 0:
        out["fp64_over_mixed_p50_latency"] = round(out["f64"]["at_rate"]["p50_ms"] / out["f32"]["at_rate"]["p50_ms"], 3)
    if out["f32"]["at_rate"]["p99_ms"] > 0:
        out["fp64_over_mixed_p99_latency"] = round(out["f64"]["at_rate"]["p99_ms"] / out["f32"]["at_rate"]["p99_ms"], 3)
    return out


if __name__ == "__main__":
    main()
