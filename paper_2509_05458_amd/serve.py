"""Served evaluation stream: many concurrent iterative solves, each a sequence
of matvecs (cfmm_eval calls) on its own resident plan.

Continuous batching on one GPU: a dispatcher admits requests in arrival order
as soon as a slot is free and the HBM budget holds the request's plan; each
slot is a worker thread with its own HIP stream, so the kernels of all
admitted requests overlap on the device while newly arrived requests wait
for the next free slot.  A request's plan (tree, lists, expansions, tables)
stays resident for all of its matvecs and is freed when the request ends.
Precision policy: the mixed near field where the tolerance is 1e-6 or looser,
FP64 otherwise.

The reference point is sequential plain-FP64 evaluation: one request at a
time on one stream, every request in FP64.  Its latencies under the same
arrivals follow from its measured service times (first come, first served).

    python -m paper_2509_05458_amd.serve --requests 64 --slots 4
"""
from __future__ import annotations

import argparse
import json
import math
import os
import queue
import sys
import threading
import time

import numpy as np

from . import Plan


def precision_for(tol: float) -> str:
    return "mixed" if tol >= 1e-6 else "fp64"


def estimate_bytes(dim: int, n: int) -> int:
    """Pre-plan HBM estimate used for admission (replaced by the plan's own
    cfmm_plan_bytes once it exists): points, sorted copies, tree, lists,
    expansions and tables, with translation scratch for 3D."""
    per_point = 1200 if dim == 2 else 2500
    return int(per_point * n + (64 << 20))


class Prepared:
    """A request with its host arrays drawn (before the clock starts)."""

    def __init__(self, req):
        self.req = req
        self.points = req.points()
        self.a, self.b = req.density_factors()


def _process(prep, precision, stream, dev, keep_last=False, on_plan=None):
    """Plan + nmat matvecs of one request on `stream`; returns (plan bytes, last result).
    on_plan(nbytes) is called once the plan exists (for memory accounting)."""
    import torch
    r = prep.req
    with torch.cuda.stream(stream):
        pts = torch.from_numpy(prep.points).to(dev)
        a = torch.from_numpy(prep.a).to(dev)
        b = torch.from_numpy(prep.b).to(dev)
        plan = Plan(pts, "helmholtz", r.kappa, r.tol, precision=precision, stream=stream.cuda_stream)
        nbytes = plan.nbytes
        if on_plan is not None:
            on_plan(nbytes)
        out = torch.empty(r.n, dtype=torch.complex128, device=dev)
        two_pi_i = 2j * math.pi
        for m in range(r.nmat):
            sig = a * torch.exp((two_pi_i * m) * b)
            plan.eval_into(sig, out)
        last = out.clone() if keep_last else None
    stream.synchronize()
    del plan
    return nbytes, last


class Server:
    def __init__(self, slots: int = 4, hbm_budget: int = 64 << 30, device: int = 0,
                 keep_results: bool = False, policy=precision_for):
        self.slots = slots
        self.budget = hbm_budget
        self.device = device
        self.keep = keep_results
        self.policy = policy

    def run(self, prepared: list, rate_scale: float = 1.0, progress=None) -> dict:
        """Serve `prepared` requests with arrivals at req.arrival * rate_scale
        seconds after the start; returns per-request records and stats.
        progress(msg), when given, is called every 64 admitted requests."""
        import torch
        dev = torch.device("cuda", self.device)
        work = queue.Queue()
        cv = threading.Condition()
        state = {"free": self.slots, "used": 0, "peak": 0}
        rec = [None] * len(prepared)
        errors = []

        def worker():
            stream = torch.cuda.Stream(device=dev)
            while True:
                item = work.get()
                if item is None:
                    return
                k, prep, reserved = item
                held = [reserved]

                def on_plan(nbytes):
                    # replace the estimate by the plan's own resident footprint
                    with cv:
                        state["used"] += nbytes - held[0]
                        state["peak"] = max(state["peak"], state["used"])
                        held[0] = nbytes
                        cv.notify_all()

                try:
                    t_start = time.perf_counter()
                    nbytes, last = _process(prep, self.policy(prep.req.tol), stream, dev, self.keep, on_plan)
                    t_end = time.perf_counter()
                    rec[k] = {"rid": prep.req.rid, "start": t_start, "end": t_end, "bytes": nbytes,
                              "result": last}
                except Exception as e:  # surfaced after the run
                    errors.append((prep.req.rid, repr(e)))
                finally:
                    with cv:
                        state["used"] -= held[0]
                        state["free"] += 1
                        cv.notify_all()

        threads = [threading.Thread(target=worker, daemon=True) for _ in range(self.slots)]
        for th in threads:
            th.start()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        admit = [0.0] * len(prepared)
        for k, prep in enumerate(prepared):
            r = prep.req
            target = t0 + r.arrival * rate_scale
            now = time.perf_counter()
            if target > now:
                time.sleep(target - now)
            est = estimate_bytes(r.dim, r.n)
            with cv:
                while state["free"] == 0 or (state["used"] > 0 and state["used"] + est > self.budget):
                    cv.wait()
                state["free"] -= 1
                state["used"] += est
                state["peak"] = max(state["peak"], state["used"])
            admit[k] = time.perf_counter()
            work.put((k, prep, est))
            if progress is not None and (k + 1) % 64 == 0:
                progress(f"admitted {k + 1}/{len(prepared)}")
        for _ in threads:
            work.put(None)
        for th in threads:
            th.join()
        if errors:
            raise RuntimeError(f"served requests failed: {errors[:3]}")
        t_end = max(x["end"] for x in rec)
        lat = np.array([rec[k]["end"] - (t0 + prepared[k].req.arrival * rate_scale)
                        for k in range(len(prepared))])
        return {"records": rec, "latency": lat, "makespan": t_end - t0, "peak_bytes": state["peak"],
                "admit_wait": np.array([admit[k] - (t0 + prepared[k].req.arrival * rate_scale)
                                        for k in range(len(prepared))])}


def sequential_service_times(prepared: list, device: int = 0, keep_results: bool = False, progress=None):
    """Plain FP64, one request at a time on one stream; service time per request.
    progress(msg), when given, is called every 64 requests."""
    import torch
    dev = torch.device("cuda", device)
    stream = torch.cuda.Stream(device=dev)
    times, results = [], []
    torch.cuda.synchronize(dev)
    for prep in prepared:
        t0 = time.perf_counter()
        _, last = _process(prep, "fp64", stream, dev, keep_results)
        times.append(time.perf_counter() - t0)
        results.append(last)
        if progress is not None and len(times) % 64 == 0:
            progress(f"sequential {len(times)}/{len(prepared)}")
    return np.array(times), results


def fcfs_latencies(arrivals: np.ndarray, service: np.ndarray):
    """Latency of each request through a single FIFO server."""
    finish = np.empty_like(service)
    t = 0.0
    for i in range(len(service)):
        t = max(t, arrivals[i]) + service[i]
        finish[i] = t
    return finish - arrivals, finish[-1] - arrivals[0]


def interactions(prepared) -> float:
    return float(sum(p.req.n * (p.req.n - 1) * p.req.nmat for p in prepared))


def serve_benchmark(nreq: int = 64, slots: int = 4, load: float = 0.8, nmax_log2: float = 18.0,
                    hbm_budget: int = 64 << 30, check: int = 8, seed: int = 4000, progress=None) -> dict:
    """Served stream against sequential plain FP64 on the same trace.

    The arrival rate is load / (mean sequential service time); sequential
    latencies come from its measured service times under those arrivals.
    `check` requests are compared served vs sequential on their last matvec.
    """
    import synth
    trace = synth.serving_trace(nreq, rate=1.0, nmax_log2=nmax_log2, seed=seed)
    prepared = [Prepared(r) for r in trace]
    # warm the library and the allocator on a small plan of each kind
    warm = [Prepared(r) for r in synth.serving_trace(4, rate=1.0, nmax_log2=11.0, seed=seed + 1)]
    sequential_service_times(warm)
    svc, seq_res = sequential_service_times(prepared, keep_results=True, progress=progress)
    mean_s = float(svc.mean())
    # unit-rate arrivals rescaled to the target load
    unit = np.array([p.req.arrival for p in prepared])
    rate_scale = mean_s / load
    arrivals = unit * rate_scale
    seq_lat, seq_span = fcfs_latencies(arrivals, svc)
    srv = Server(slots=slots, hbm_budget=hbm_budget, keep_results=True).run(prepared, rate_scale=rate_scale,
                                                                           progress=progress)
    lat = srv["latency"]
    diffs = []
    for k in range(min(check, nreq)):
        a = srv["records"][k]["result"].cpu().numpy()
        b = seq_res[k].cpu().numpy()
        diffs.append(float(np.linalg.norm(a - b) / np.linalg.norm(b)))
    # both results are within tol of the exact sum, so they differ by at most 2 tol
    ok = all(d <= 2.0 * prepared[k].req.tol for k, d in enumerate(diffs))
    inter = interactions(prepared)
    nmat = sum(p.req.nmat for p in prepared)
    # saturation throughput: every request present at t = 0
    burst = Server(slots=slots, hbm_budget=hbm_budget).run(prepared, rate_scale=0.0, progress=progress)
    seq_total = float(svc.sum())
    return {
        "requests": nreq, "slots": slots, "load": load, "matvecs": nmat,
        "arrival_rate_per_s": 1.0 / rate_scale, "mean_sequential_service_s": mean_s,
        "served": {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                   "makespan_s": srv["makespan"], "matvecs_per_s": nmat / srv["makespan"],
                   "interactions_per_s": inter / srv["makespan"], "peak_admitted_bytes": int(srv["peak_bytes"])},
        "sequential_fp64": {"p50_ms": float(np.percentile(seq_lat, 50) * 1e3),
                            "p99_ms": float(np.percentile(seq_lat, 99) * 1e3),
                            "makespan_s": float(seq_span), "matvecs_per_s": nmat / float(seq_span),
                            "interactions_per_s": inter / float(seq_span)},
        "burst": {"served_makespan_s": burst["makespan"], "sequential_fp64_makespan_s": seq_total,
                  "served_matvecs_per_s": nmat / burst["makespan"], "sequential_matvecs_per_s": nmat / seq_total,
                  "served_interactions_per_s": inter / burst["makespan"],
                  "sequential_interactions_per_s": inter / seq_total},
        "served_vs_sequential_rel_diff": diffs, "within_tol": ok,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--nmax-log2", type=float, default=18.0)
    ap.add_argument("--hbm-budget-gib", type=float, default=64.0)
    a = ap.parse_args(argv)
    def progress(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    res = serve_benchmark(a.requests, a.slots, a.load, a.nmax_log2, int(a.hbm_budget_gib * (1 << 30)),
                          progress=progress)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    main()
