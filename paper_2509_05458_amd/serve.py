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

Each request is an iterative solve: its matvecs run one after another, the
density of matvec m + 1 formed from the result of matvec m by an Arnoldi step
(orthogonalised against the request's earlier densities and normalised, as
GMRES does), with a host wait on each step's norm.  So a request's matvecs
never overlap each other; requests overlap one another.

The reference point is sequential plain-FP64 evaluation: the same arrival
trace replayed through one slot on one stream, every request in FP64
(measured, not modelled).

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
    """Plan + nmat dependent matvecs of one request on `stream`.

    Matvec 0 takes the request's seeded density a (normalised); matvec m + 1
    takes the Arnoldi vector of matvec m's result w = A v_m: w minus its
    projections on v_0 .. v_m, divided by its norm, which the host reads
    (the wait a GMRES iteration makes).  Returns (plan bytes, (last density,
    last result) or None).  on_plan(nbytes) is called once the plan exists
    (for memory accounting)."""
    import torch
    r = prep.req
    with torch.cuda.stream(stream):
        pts = torch.from_numpy(prep.points).to(dev)
        a = torch.from_numpy(prep.a).to(dev)
        plan = Plan(pts, "helmholtz", r.kappa, r.tol, precision=precision, stream=stream.cuda_stream)
        nbytes = plan.nbytes
        if on_plan is not None:
            on_plan(nbytes)
        V = torch.empty((r.nmat, r.n), dtype=torch.complex128, device=dev)
        out = torch.empty(r.n, dtype=torch.complex128, device=dev)
        V[0] = a / torch.linalg.vector_norm(a)
        for m in range(r.nmat):
            plan.eval_into(V[m], out)
            if m + 1 == r.nmat:
                break
            h = torch.mv(V[: m + 1].conj(), out)            # projections on v_0 .. v_m
            w = out - torch.mv(V[: m + 1].transpose(0, 1), h)
            nrm = float(torch.linalg.vector_norm(w))        # host wait
            V[m + 1] = w / nrm
        last = (V[r.nmat - 1].clone(), out.clone()) if keep_last else None
    plan.sync()
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


def sequential_fp64(slots_run_kwargs=None):
    """The sequential plain-FP64 reference: one slot (one stream), FP64 for
    every request."""
    return Server(slots=1, policy=lambda tol: "fp64", **(slots_run_kwargs or {}))


def interactions(prepared) -> float:
    return float(sum(p.req.n * (p.req.n - 1) * p.req.nmat for p in prepared))


def torch_norm(x) -> float:
    import torch
    return float(torch.linalg.vector_norm(x))


def _reference(prep, sig):
    """The request's geometry evaluated for density sig by a plain FP64 plan
    at tol 1e-10, on the current stream."""
    import torch
    r = prep.req
    pts = torch.from_numpy(prep.points).to(sig.device)
    plan = Plan(pts, "helmholtz", r.kappa, 1e-10, precision="fp64")
    u = plan(sig)
    plan.sync()
    torch.cuda.synchronize(sig.device)
    return u


def _stats(run, nmat, inter):
    lat = run["latency"]
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "makespan_s": run["makespan"], "matvecs_per_s": nmat / run["makespan"],
            "interactions_per_s": inter / run["makespan"], "peak_admitted_bytes": int(run["peak_bytes"])}


def serve_benchmark(nreq: int = 64, slots: int = 4, load: float = 0.8, nmax_log2: float = 18.0,
                    hbm_budget: int = 64 << 30, check: int = 8, seed: int = 4000, progress=None,
                    nmat: int = 20) -> dict:
    """Served stream against sequential plain FP64 on the same arrival trace.

    1. Sequential FP64 with every request present at t = 0 gives the mean
       sequential service time S and the sequential saturation throughput.
    2. Arrivals are Poisson at load / S.  The trace is replayed through the
       server (slots, mixed where tol >= 1e-6) and through one FP64 slot;
       both latencies are measured (arrival to the last matvec's result).
    3. The served run with every request present at t = 0 gives the served
       saturation throughput.
    `check` requests' last served matvecs are compared with a plain FP64
    evaluation at tol 1e-10 of the same density.
    """
    import synth
    trace = synth.serving_trace(nreq, rate=1.0, nmax_log2=nmax_log2, seed=seed, nmat=nmat)
    prepared = [Prepared(r) for r in trace]
    # warm the library and the allocator on a small plan of each kind
    warm = [Prepared(r) for r in synth.serving_trace(4, rate=1.0, nmax_log2=11.0, seed=seed + 1, nmat=2)]
    sequential_fp64().run(warm, rate_scale=0.0)
    seq_burst = sequential_fp64({"keep_results": True}).run(prepared, rate_scale=0.0, progress=progress)
    svc = np.array([r["end"] - r["start"] for r in seq_burst["records"]])
    mean_s = float(svc.mean())
    rate_scale = mean_s / load                  # unit-rate arrivals rescaled to the target load
    srv = Server(slots=slots, hbm_budget=hbm_budget, keep_results=True).run(prepared, rate_scale=rate_scale,
                                                                           progress=progress)
    seq = sequential_fp64().run(prepared, rate_scale=rate_scale, progress=progress)
    # accuracy of the served results: each checked request's last density is
    # evaluated again by a plain FP64 plan at tol 1e-10 (far tighter than
    # any request's tolerance), and the served result must agree within tol
    diffs = []
    for k in range(min(check, nreq)):
        sig, u = srv["records"][k]["result"]
        ref = _reference(prepared[k], sig)
        diffs.append(float(torch_norm(u - ref) / torch_norm(ref)))
    ok = all(d <= prepared[k].req.tol + 1e-10 for k, d in enumerate(diffs))
    inter = interactions(prepared)
    nmv = sum(p.req.nmat for p in prepared)
    burst = Server(slots=slots, hbm_budget=hbm_budget).run(prepared, rate_scale=0.0, progress=progress)
    return {
        "requests": nreq, "slots": slots, "load": load, "matvecs": nmv, "nmax_log2": nmax_log2,
        "arrival_rate_per_s": 1.0 / rate_scale, "mean_sequential_service_s": mean_s,
        "served": _stats(srv, nmv, inter),
        "sequential_fp64": _stats(seq, nmv, inter),
        "burst": {"served_makespan_s": burst["makespan"], "sequential_fp64_makespan_s": seq_burst["makespan"],
                  "served_matvecs_per_s": nmv / burst["makespan"],
                  "sequential_matvecs_per_s": nmv / seq_burst["makespan"],
                  "served_interactions_per_s": inter / burst["makespan"],
                  "sequential_interactions_per_s": inter / seq_burst["makespan"]},
        "served_vs_fp64_reference_rel_diff": diffs, "within_tol": ok,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--nmax-log2", type=float, default=18.0)
    ap.add_argument("--hbm-budget-gib", type=float, default=64.0)
    ap.add_argument("--matvecs", type=int, default=20)
    a = ap.parse_args(argv)
    def progress(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    res = serve_benchmark(a.requests, a.slots, a.load, a.nmax_log2, int(a.hbm_budget_gib * (1 << 30)),
                          progress=progress, nmat=a.matvecs)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    main()
