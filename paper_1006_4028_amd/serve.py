"""Continuous-batching server for propagator requests on resident gauge fields.

Each resident field has a `Lattice` (its own HIP stream) and a `Batch` of
slots driven by a worker thread; the threads release the GIL inside the
library, so the work of different fields overlaps on the GPU.  A request asks
for `ncols` point-source columns at timeslice x0 with mass M and a distance
profile alpha0; it is admitted when its field's batch has `ncols` free slots
and, if its mass is new on that field, when the HBM budget still holds one
more per-mass inverse clover.  Requests that arrive while others run join the
running batch at the next step; finished columns leave it.  Latency is
measured from arrival to the completion of the request's last column.
"""
import dataclasses
import queue
import threading
import time

import numpy as np

from . import Batch, Lattice, footprint_bytes


@dataclasses.dataclass
class Request:
    rid: int
    field: str
    M: float
    alpha0: float
    ncols: int
    x0: int
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    status: str = "queued"
    cpp: np.ndarray = None
    infos: list = dataclasses.field(default_factory=list)
    _left: int = 0


def profile(T, alpha0, x0):
    """alpha(x0') = exp(alpha0 min(t, T - t)), t = (x0' - x0) mod T."""
    t = (np.arange(T) - x0) % T
    return np.exp(alpha0 * np.minimum(t, T - t).astype(np.float64))


def point_columns(dims, x0, ncols):
    """The first ncols spin-colour unit sources at (x0, 0, 0, 0), host layout."""
    eta = np.zeros((ncols,) + tuple(dims) + (4, 3), dtype=np.complex128)
    for c in range(ncols):
        eta[(c, x0, 0, 0, 0, c // 3, c % 3)] = 1.0
    return eta


class FieldWorker(threading.Thread):
    def __init__(self, name, lattice, nslots, precision, r, max_iter, k, budget, mem_lock, mem_state):
        super().__init__(daemon=True)
        self.fname = name
        self.L = lattice
        self.batch = Batch(lattice, nslots, precision)
        self.q = queue.Queue()
        self.pending = []
        self.running = {}
        self.r, self.max_iter, self.k = r, max_iter, k
        self.masses = set()
        self.budget, self.mem_lock, self.mem = budget, mem_lock, mem_state
        self.mass_bytes = footprint_bytes(lattice.dims, 0, precision, 1) - footprint_bytes(lattice.dims, 0, precision, 0)
        self.closing = False
        self.error = None
        self.steps = 0
        self.occupancy = []

    def _try_admit(self, req):
        st = self.batch.status()
        if req.ncols > self.batch.nslots:
            req.status = "rejected_slots"
            return True
        if st["free"] < req.ncols:
            return False
        if req.M not in self.masses:
            with self.mem_lock:
                if self.mem["used"] + self.mass_bytes > self.budget:
                    req.status = "rejected_memory"
                    return True
                self.mem["used"] += self.mass_bytes
            self.masses.add(req.M)
        eta_t = self.L.point_sources((req.x0, 0, 0, 0), 0, req.ncols)
        slots = self.batch.admit(eta_t, None, M=req.M, alpha=profile(self.L.T, req.alpha0, req.x0), r=self.r,
                                 max_iter=self.max_iter, x0_src=req.x0, tag=req.rid)
        assert slots is not None
        req.t_admit = time.perf_counter()
        req.status = "running"
        req._left = req.ncols
        req.cpp = np.zeros(self.L.T)
        self.running[req.rid] = req
        return True

    def run(self):
        try:
            while True:
                while True:
                    try:
                        self.pending.append(self.q.get_nowait())
                    except queue.Empty:
                        break
                while self.pending and self._try_admit(self.pending[0]):
                    self.pending.pop(0)
                if self.running:
                    st = self.batch.status()
                    self.occupancy.append(st["running"] / self.batch.nslots)
                    self.batch.step(self.k)
                    self.steps += 1
                    for res in self.batch.harvest():
                        req = self.running[res["tag"]]
                        req.cpp += res["cpp"]
                        req.infos.append(res["info"])
                        req._left -= 1
                        if req._left == 0:
                            req.t_done = time.perf_counter()
                            ok = all(i["status"] == 0 for i in req.infos)
                            req.status = "done" if ok else "failed"
                            self.batch.release(req.rid)
                            del self.running[req.rid]
                elif self.closing and not self.pending and self.q.empty():
                    break
                else:
                    try:
                        self.pending.append(self.q.get(timeout=0.001))
                    except queue.Empty:
                        pass
        except Exception as e:  # surfaced by Server.run
            self.error = e


class Server:
    """fields: {name: (dims, U, csw)}; one worker thread and batch per field."""

    def __init__(self, fields, nslots=12, precision="f32", r=1e-10, max_iter=20000, k=4, hbm_budget=None):
        self.lattices = {}
        self.workers = {}
        self.mem_lock = threading.Lock()
        self.mem = {"used": 0}
        budget = hbm_budget if hbm_budget is not None else float("inf")
        for name, (dims, U, csw) in fields.items():
            L = Lattice(dims)
            L.set_gauge(U)
            L.set_clover(csw)
            self.lattices[name] = L
            self.mem["used"] += footprint_bytes(dims, nslots, precision, 0)
            self.workers[name] = FieldWorker(name, L, nslots, precision, r, max_iter, k, budget, self.mem_lock,
                                             self.mem)

    def run(self, requests, progress=0):
        """Submit the requests at their arrival offsets (seconds, request.t_arrival
        relative to the start); return the requests when all are finished.
        progress > 0 logs the submitted and finished counts to stderr every
        `progress` submissions and whenever the finished count changes while
        the last requests drain (checked every 10 s)."""
        import sys
        for w in self.workers.values():
            w.start()
        t0 = time.perf_counter()
        reqs = sorted(requests, key=lambda q: q.t_arrival)

        def finished():
            return sum(q.status not in ("", "queued", "running") for q in reqs)

        for k, req in enumerate(reqs, 1):
            delay = t0 + req.t_arrival - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            req.t_arrival = time.perf_counter()
            self.workers[req.field].q.put(req)
            if progress and k % progress == 0:
                print(f"  {k}/{len(reqs)} submitted, {finished()} finished", file=sys.stderr, flush=True)
        for w in self.workers.values():
            w.closing = True
        last = -1
        for w in self.workers.values():
            while w.is_alive():
                w.join(timeout=10.0)
                n = finished()
                if progress and n != last:
                    print(f"  draining: {n}/{len(reqs)} finished", file=sys.stderr, flush=True)
                    last = n
            if w.error:
                raise w.error
        self.t_start, self.t_end = t0, time.perf_counter()
        return requests

    def close(self):
        for w in self.workers.values():
            w.batch.close()
        for L in self.lattices.values():
            L.close()


def poisson_requests(n, rate, fields, T_of, seed, masses=(0.01, 0.05, 0.2, 0.5), alpha0s=(0.0, 0.1, 0.4),
                     max_cols=12):
    """n requests with exponential inter-arrival times at `rate` per second, each
    drawing field, M, alpha0, the column count 1..max_cols and x0 uniformly."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    names = list(fields)
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        f = names[rng.integers(len(names))]
        out.append(Request(rid=i, field=f, M=float(rng.choice(masses)), alpha0=float(rng.choice(alpha0s)),
                           ncols=int(rng.integers(1, max_cols + 1)), x0=int(rng.integers(T_of[f])), t_arrival=t))
    return out


def summarize(server, reqs):
    done = [q for q in reqs if q.status == "done"]
    lat = np.array([q.t_done - q.t_arrival for q in done]) if done else np.zeros(1)
    cols = sum(q.ncols for q in done)
    span = server.t_end - server.t_start
    occ = [o for w in server.workers.values() for o in w.occupancy]
    return dict(requests=len(reqs), done=len(done), rejected=sum(q.status.startswith("rejected") for q in reqs),
                failed=sum(q.status == "failed" for q in reqs), solves=cols, seconds=span,
                solves_per_s=cols / span if span > 0 else 0.0, p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), mean_slot_occupancy=float(np.mean(occ)) if occ else 0.0)


def sweep(loads=(0.5, 0.8, 1.0, 1.2), requests=150, r=1e-10, seed=2024, nslots=24, out=None, progress=0):
    """The served-stream measurement: resident 16^3x32 and 24^3x48 fields, the
    FP64-inner capacity measured first (a saturating stream), then Poisson
    streams at the given fractions of that capacity, FP32 and FP64 inner, each
    reporting solves/s and p50/p99 latency.  Returns the list of records."""
    import json
    import synth
    fields = {}
    for name in ("su3_16c32", "su3_24c48"):
        cfg = synth.config(name)
        fields[name] = (cfg["dims"], synth.gauge_su3(cfg["dims"], cfg["eps"], cfg["seed"]), cfg["csw"])
    T_of = {k: v[0][0] for k, v in fields.items()}
    recs = []

    def run(prec, rate, n):
        reqs = poisson_requests(n, rate, fields, T_of, seed=seed)
        srv = Server(fields, nslots=nslots, precision=prec, r=r, max_iter=20000, k=4)
        try:
            s = summarize(srv, srv.run(reqs, progress=progress))
        finally:
            srv.close()
        rec = dict(precision=prec, rate_per_s=rate, r=r, **s)
        print(json.dumps(rec), flush=True)
        if out:
            out.write(json.dumps(rec) + "\n")
            out.flush()
        return rec

    cap = run("f64", 1000.0, max(40, requests // 3))  # every request at once: the capacity
    mean_cols = cap["solves"] / max(cap["done"], 1)
    cap_req = cap["solves_per_s"] / mean_cols
    recs.append(dict(cap, kind="capacity"))
    for f in loads:
        for prec in ("f32", "f64"):
            rec = run(prec, f * cap_req, requests)
            rec["load"] = f
            recs.append(rec)
    return recs


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="served-stream load sweep (one GPU)")
    ap.add_argument("--requests", type=int, default=150)
    ap.add_argument("--r", type=float, default=1e-10)
    ap.add_argument("--loads", default="0.5,0.8,1.0,1.2")
    ap.add_argument("--out", default=None, help="also append the JSON records to this file")
    ap.add_argument("--progress", type=int, default=0, help="log progress every N submitted requests")
    a = ap.parse_args()
    f = open(a.out, "a") if a.out else None
    sweep(tuple(float(x) for x in a.loads.split(",")), a.requests, a.r, out=f, progress=a.progress)
