#!/usr/bin/env python3
"""Benchmark of the complex-coordinate FMM hot path on one MI355X.

A step is one cfmm_eval on a warm plan (density gather, P2M, M2M, M2L+P2L,
L2L, L2P+M2P, P2P, scatter) for one fresh density vector; the plan (points,
Morton sort, tree, centres, lists, expansion lengths) is built once before
timing, as in the iterative solves the method serves, and its time is
reported separately.

Workload (default, --workload c2, the largest single-GPU configuration): 3D
Laplace single layer, N = 1448^2 = 2,096,704 points on the complexified plane
(s + i psi(s), t + i psi(t), 0.3 exp(-(s^2 + t^2))), tolerance 1e-6, FP64.
--workload c1: 2D Helmholtz, N = 2^20 points on the complexified curve
(t + i psi(t), 0.2 exp(-t^2)) scaled by 0.1, kappa = 100; c3: 3D Helmholtz on
the 1000^2 plane with bumps, kappa = 20 * 2 pi / 12.

Prints one JSON line.  metric: N^2-equivalent interactions per second,
N (N - 1) / t_eval, with a roofline block for the dominant kernel, the near
field (HIP events on the plan's stream over the timed steps; for 3D Laplace
the M2L translations are reported beside it), the oracle's direct sum on the
host's cores as cpu_baseline, and a serving block: a seeded stream of
GMRES-like requests served with overlap and memory admission against the same
trace replayed sequentially in plain FP64.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic flops of one near-field interaction G(x_i, y_j) sigma_j, counting
# add/mul as 1, FMA as 2 and each sqrt, divide, exp or sincos as 1:
#  * 2D Helmholtz in the small-argument regime of the C1 curve (|kappa r| < 0.1):
#    squared complex distance 15, complex log 10, five series terms of J0 and Y0
#    at 12 each, assembly 8, complex multiply-accumulate 8;
#  * 3D Laplace: squared complex distance 18, principal root and 1/r 9,
#    complex multiply-accumulate 8;
#  * 3D Helmholtz: as 3D Laplace plus e^{i kappa r} (exp, sincos, 6) and the
#    complex product with 1/r (6).
# Of each figure, 8 flops are the complex multiply-accumulate into one target;
# the rest is the kernel evaluation, which the 2D near field shares between
# the two directions of a symmetric pair (cfmm_plan_near_work).
MAC_FLOPS = 8.0
WORKLOADS = {
    # name: (config index, dim, kernel, default tol, P2P kernel, flops per interaction)
    "c1": (1, 2, "helmholtz", 1e-6, "P2P stage: k_h2d_p2p_sym + k_h2d_p2p_diag + k_h2d_p2p_row + k_h2d_p2p_final", 100.0),
    "c2": (2, 3, "laplace", 1e-6, "P2P stage: k_near3_pair + k_near3_diag + k_near3_final", 35.0),
    "c3": (3, 3, "helmholtz", 1e-6, "P2P stage: k_near3_pair + k_near3_diag + k_near3_final", 47.0),
}
PEAK_FP64_VALU = 78.6e12          # 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
PEAK_FP32_VALU = 157.3e12
METRIC = "N\u00b2-equiv interactions/s at 1e-6 rel err; served p50/p99 latency vs plain"


TRAFFIC_PROFILES = {
    # FP64 workload: counter summary of its P2P kernels (calibrated HBM bytes per launch)
    "c2_m2l": "profiles/laplace3d_n2m_m2l_traffic.md",
    "c1": "profiles/helmholtz2d_n1m_p2p_traffic.md",
    "c2": "profiles/laplace3d_n2m_p2p_traffic.md",
    "c3": "profiles/helmholtz3d_n1m_p2p_traffic.md",
}


def measured_traffic(workload: str):
    """HBM bytes per launch of the workload's P2P kernel from the committed
    counter summary, or None when there is none or when the kernel sources
    have changed since the counters were taken."""
    import hashlib
    path = TRAFFIC_PROFILES.get(workload)
    if not path or not os.path.exists(os.path.join(ROOT, path)):
        return None
    fields = {}
    for line in open(os.path.join(ROOT, path)):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for src in fields["kernel_sources"].split(","):
            h.update(open(os.path.join(ROOT, src.strip()), "rb").read())
        if h.hexdigest() != fields["kernel_source_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--cpu-targets", type=int, default=96, help="least oracle targets of the CPU leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 512 MiB device copy (counter calibration for HBM traffic)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving block")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision block")
    ap.add_argument("--no-cpu-fmm", action="store_true", help="skip the CPU FMM reference")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-nmax-log2", type=float, default=16.0)
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU sharding is a design "
              "(see the sharding section of the design notes), not a runnable path.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2509_05458_amd as cf
    import synth

    ci, dim, kern, tol0, p2p_kernel, p2p_flops_unit = WORKLOADS[a.workload]
    tol = a.tol or tol0
    cfg = synth.make_config(ci, n=a.n or None)
    n = cfg.n
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(cfg.points).to(dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = cf.Plan(pts, kern, cfg.kappa, tol, precision=a.precision, leaf_size=a.leaf,
                   stream=stream.cuda_stream)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    # the plan's own phase clock: keys and sort, topology and lists (both on
    # the device), centres and expansion lengths, tables and work lists (host),
    # the geometry check (device)
    plan_phases = {k: round(v, 3) for k, v in plan.timing().items()}
    info = plan.info()
    # fresh seeded densities per step, resident in HBM before timing
    nsig = max(1, min(4, a.steps))
    sigs = [torch.from_numpy(synth.density(n, 2000 + ci + 17 * k)).to(dev) for k in range(nsig)]
    out = torch.empty_like(sigs[0])
    for w in range(a.warmup):
        plan.eval_into(sigs[w % nsig], out)
    torch.cuda.synchronize()
    # timed region: back-to-back evaluations; HIP events on the plan's stream
    # bracket the dominant stage of each one, the near field on every
    # workload (profiling mode 2); the M2L translations (mode 3) are
    # bracketed over a few evaluations after it
    plan.set_profiling(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        plan.eval_into(sigs[s % nsig], out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ring_tot, ring_cnt = plan.ring_ms()
    # the other stage's ring over a few more evaluations (after the timed region)
    nside = max(1, min(a.steps, 5))
    plan.set_profiling(3)
    for s in range(nside):
        plan.eval_into(sigs[s % nsig], out)
    torch.cuda.synchronize()
    side_tot, side_cnt = plan.ring_ms()
    plan.set_profiling(0)
    near_ms, m2l_ms = ring_tot / max(1, ring_cnt), side_tot / max(1, side_cnt)
    ms_per_step = dt * 1e3 / a.steps
    pairs = n * (n - 1)
    value = pairs / (ms_per_step * 1e-3)
    # stage split, after the timed region: every stage bracketed, one
    # evaluation at a time
    nsplit = max(1, min(a.steps, 5))
    plan.set_profiling(1)
    stage_tot = {k: 0.0 for k in cf.STAGES}
    for s in range(nsplit):
        plan.eval_into(sigs[s % nsig], out)
        torch.cuda.synchronize()
        for k, v in plan.stage_ms().items():
            stage_tot[k] += v
    plan.set_profiling(0)
    stage_avg = {k: v / nsplit for k, v in stage_tot.items()}
    # the output checked below is that of the last timed step's density
    plan.eval_into(sigs[(a.steps - 1) % nsig], out)
    torch.cuda.synchronize()

    if a.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    u_gpu = out.cpu().numpy()
    sig_last = sigs[(a.steps - 1) % nsig].cpu().numpy()

    # the same workload through the mixed-precision path (tol >= 1e-6 only),
    # timed the same way, for the north-star's second precision form
    mixed = None
    if a.precision == "fp64" and not a.no_mixed and tol >= 1e-6 and dim == 3:
        mplan = cf.Plan(pts, kern, cfg.kappa, tol, precision="mixed", leaf_size=a.leaf,
                        stream=stream.cuda_stream)
        for w in range(a.warmup):
            mplan.eval_into(sigs[w % nsig], out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(a.steps):
            mplan.eval_into(sigs[s_ % nsig], out)
        torch.cuda.synchronize()
        mdt = (time.perf_counter() - t0) * 1e3 / a.steps
        mplan.eval_into(sigs[(a.steps - 1) % nsig], out)
        torch.cuda.synchronize()
        mixed = {"ms_per_step": mdt, "value": pairs / (mdt * 1e-3), "dtype": "f32+f64",
                 "u": out.cpu().numpy()}
        del mplan
    nw = plan.near_work()
    p2p_flops = (p2p_flops_unit - MAC_FLOPS) * nw["evaluations"] + MAC_FLOPS * nw["interactions"]
    peak = PEAK_FP64_VALU if a.precision == "fp64" else PEAK_FP32_VALU
    p2p_block = {
        "kernel": p2p_kernel, "bound": "alu", "achieved": p2p_flops / (near_ms * 1e-3) / 1e12,
        "peak": peak / 1e12, "unit": "TFLOP/s", "frac": p2p_flops / (near_ms * 1e-3) / peak,
        "traffic": measured_traffic(a.workload) if a.precision == "fp64" else None,
        "flops_per_interaction": p2p_flops_unit, "ms_per_launch_set": near_ms,
        "near_interactions": nw["interactions"], "near_evaluations": nw["evaluations"],
    }
    roof = dict(p2p_block)
    if dim == 3 and kern == "laplace":
        # the M2L translations: point-and-shoot pairs (k_l3d_m2l_pns: four
        # real rotations per degree, the coaxial shift and the diagonal
        # phases) and direct-form pairs (k_l3d_m2l: (P+1)^2 (Ps+1)^2 complex
        # multiply-adds); algorithmic flops of each from cfmm_plan_m2l_work
        P = info["max_p"]
        mw = plan.m2l_work()
        m2l_flops = float(mw["direct_flops"] + mw["pns_flops"])
        mixed_direct = a.precision == "mixed" and P <= 16 and mw["direct_pairs"] > 0
        m2l_peak = PEAK_FP64_VALU
        m2l_kern = ("k_l3d_m2l_pns + " if mw["pns_pairs"] else "") + ("k_l3d_m2l_f32" if mixed_direct else "k_l3d_m2l")
        roof["m2l"] = {
            "kernel": m2l_kern,
            "bound": "alu", "achieved": m2l_flops / (m2l_ms * 1e-3) / 1e12, "peak": m2l_peak / 1e12,
            "unit": "TFLOP/s", "frac": m2l_flops / (m2l_ms * 1e-3) / m2l_peak,
            "traffic": measured_traffic("c2_m2l") if (a.precision == "fp64" and a.workload == "c2") else None,
            "flops_per_pair_mean": m2l_flops / max(1, info["m2l_pairs"]), "pairs": info["m2l_pairs"],
            "pns_pairs": mw["pns_pairs"], "direct_pairs": mw["direct_pairs"],
            "pns_flops": mw["pns_flops"], "direct_flops": mw["direct_flops"],
            "ms_per_launch": m2l_ms,
        }
    else:
        roof["m2l_ms"] = m2l_ms
    names = {"c1": f"2D Helmholtz single layer, N={n} complexified curve (C0 curve scaled 0.1), "
                   f"kappa={cfg.kappa}, tol={tol}, targets=sources",
             "c2": f"3D Laplace single layer, N={n} complexified plane ({cfg.meta.get('grid')}^2 grid), "
                   f"tol={tol}, targets=sources",
             "c3": f"3D Helmholtz single layer, N={n} complexified plane with 8 bumps "
                   f"({cfg.meta.get('grid')}^2 grid), kappa={cfg.kappa:.4f} (20 wavelengths), tol={tol}, "
                   f"targets=sources"}
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": names[a.workload],
            "n": n, "kappa": cfg.kappa, "tol": tol, "precision": a.precision,
            "leaf_size": info["leaf_size"], "separation": info["separation"],
            "top_level": info["top_level"], "levels": info["nlevels"], "max_p": info["max_p"],
            "p2p_pairs": info["p2p_pairs"], "m2l_pairs": info["m2l_pairs"],
            "boxes": info["nbox"], "leaves": info["nleaf"], "list3": info["n_list3"], "list4": info["n_list4"],
            "plan_ms": plan_ms, "plan_phases_ms": plan_phases, "stage_ms": stage_avg,
            "step": "one cfmm_eval on a warm plan",
        },
        "roofline": roof,
    }
    if not a.no_cpu:
        # cpu_baseline leg: the oracle's direct FP64 sum on the host's cores at
        # seeded sampled targets, sized to about 12 s of CPU work (at most the
        # 4096 oracle targets of the configuration); its output also gives the
        # sampled error of the timed evaluation
        import oracle
        cores = len(os.sched_getaffinity(0))
        pool = cfg.oracle_targets
        t0 = time.perf_counter()
        oracle.direct_self(dim, kern, cfg.kappa, cfg.points, sig_last, targets=pool[:16], nthreads=cores)
        per = (time.perf_counter() - t0) / 16
        k = int(min(len(pool), max(a.cpu_targets, 12.0 / max(per, 1e-9))))
        ct = pool[:k]
        t0 = time.perf_counter()
        u0 = oracle.direct_self(dim, kern, cfg.kappa, cfg.points, sig_last, targets=ct, nthreads=cores)
        cdt = time.perf_counter() - t0
        res["cpu_baseline"] = {
            "value": len(ct) * (n - 1) / cdt,
            "unit": "interactions/s",
            "cores": cores,
            "kind": "oracle",
            "sample": f"{len(ct)} seeded targets x all {n} sources, FP64 direct sum ({cdt:.1f} s)",
        }
        res["config"]["rel_l2_err_sampled"] = oracle.rel_l2(u_gpu[ct], u0)
        res["config"]["rel_err_paper_sampled"] = float(np.linalg.norm(u_gpu[ct] - u0) /
                                                       (np.linalg.norm(u0) + np.linalg.norm(sig_last[ct])))
        res["config"]["err_targets"] = int(len(ct))
        if mixed is not None:
            mixed["rel_l2_err_sampled"] = oracle.rel_l2(mixed["u"][ct], u0)
        if a.workload == "c2" and not a.no_cpu_fmm:
            # the CPU FMM reference: the same method and tolerance on the host's
            # cores, on the whole workload (one evaluation, after its plan)
            import cpu_ref
            uc, (cplan, ceval) = cpu_ref.fmm3d_laplace(cfg.points, sig_last, tol, leaf_size=info["leaf_size"],
                                                       sep=info["separation"], nthreads=cores)
            res["cpu_fmm"] = {
                "value": pairs / ceval, "unit": "interactions/s", "cores": cores, "kind": "cpu FMM reference",
                "eval_s": ceval, "plan_s": cplan, "rel_l2_err_sampled": oracle.rel_l2(uc[ct], u0),
                "sample": f"the whole workload, N={n}, tol={tol}, one evaluation",
            }
    if mixed is not None:
        mixed.pop("u")
        res["mixed_precision"] = mixed
    if not a.no_serve:
        del plan, sigs, out, pts
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        from paper_2509_05458_amd import serve
        sv = serve.serve_benchmark(nreq=a.serve_requests, slots=4, load=0.8,
                                   nmax_log2=a.serve_nmax_log2, check=4,
                                   progress=lambda m: print(f"[bench serve] {m}", file=sys.stderr, flush=True))
        res["serving"] = {
            "trace": (f"{sv['requests']} seeded requests (trace seed 4000), Poisson arrivals at load 0.8 of the "
                      f"sequential service rate, N log-uniform in [2^10, 2^{a.serve_nmax_log2:g}], 2D/3D "
                      f"Helmholtz, kappa in [1, 200], tol in {{1e-4, 1e-6, 1e-10}}, {sv['matvecs'] // sv['requests']}"
                      f" dependent (Arnoldi) matvecs each"),
            "slots": sv["slots"], "arrival_rate_per_s": sv["arrival_rate_per_s"],
            "served": {k: sv["served"][k] for k in ("p50_ms", "p99_ms", "matvecs_per_s", "makespan_s")},
            "sequential_fp64": {k: sv["sequential_fp64"][k] for k in ("p50_ms", "p99_ms", "matvecs_per_s",
                                                                     "makespan_s")},
            "saturation_matvecs_per_s": {"served": sv["burst"]["served_matvecs_per_s"],
                                         "sequential_fp64": sv["burst"]["sequential_matvecs_per_s"]},
            "within_tol": sv["within_tol"],
            "max_rel_diff_vs_fp64_reference": max(sv["served_vs_fp64_reference_rel_diff"]),
        }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
