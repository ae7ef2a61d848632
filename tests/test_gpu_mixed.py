"""GPU parity of the mixed-precision path (FP32 near field with FP64-formed
differences and FP64 tile sums) against the FP64 oracle; every case prints
its relative l2 error next to the FP64 plan's."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2509_05458_amd as cf  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def _run(pts, sig, kernel, kappa, tol, precision, leaf=0):
    print(f"[gpu] mixed-test plan n={pts.shape[0]} {kernel} kappa={kappa:.4g} tol={tol} {precision}", flush=True)
    plan = cf.Plan(torch.from_numpy(pts).cuda(), kernel, kappa, tol, precision=precision, leaf_size=leaf)
    u = plan(torch.from_numpy(sig).cuda())
    torch.cuda.synchronize()
    assert plan.info()["precision"] == (1 if precision == "mixed" else 0)
    return u.cpu().numpy()


@pytest.mark.parametrize("ci,m,kernel,kappa", [(2, 48, "laplace", 0.0), (3, 56, "helmholtz", synth.KAPPA_C3)])
def test_3d_mixed_family_parity(ci, m, kernel, kappa):
    cfg = synth.make_config(ci, n=m * m)
    u0 = oracle.direct_self(3, kernel, kappa, cfg.points, cfg.sigma, nthreads=NTHREADS)
    um = _run(cfg.points, cfg.sigma, kernel, kappa, 1e-6, "mixed", 32)
    ud = _run(cfg.points, cfg.sigma, kernel, kappa, 1e-6, "fp64", 32)
    em, ed = oracle.rel_l2(um, u0), oracle.rel_l2(ud, u0)
    print(f"[gpu] {kernel} m={m}: mixed rel_l2={em:.3e}  fp64 rel_l2={ed:.3e}", flush=True)
    assert em <= 1e-6


def test_2d_mixed_parity():
    cfg = synth.make_config(1, n=1 << 14)
    tg = cfg.oracle_targets[:512]
    u0 = oracle.direct_self(2, "helmholtz", cfg.kappa, cfg.points, cfg.sigma, targets=tg, nthreads=NTHREADS)
    um = _run(cfg.points, cfg.sigma, "helmholtz", cfg.kappa, 1e-6, "mixed")
    em = oracle.rel_l2(um[tg], u0)
    print(f"[gpu] 2D mixed rel_l2={em:.3e}", flush=True)
    assert em <= 1e-6


@pytest.mark.parametrize("ci,kernel", [(3, "helmholtz"), (2, "laplace")])
def test_full_size_mixed_sampled_parity(ci, kernel):
    cfg = synth.make_config(ci, n_oracle=1024)
    um = _run(cfg.points, cfg.sigma, kernel, cfg.kappa, 1e-6, "mixed")
    tg = cfg.oracle_targets
    u0 = oracle.direct_self(3, kernel, cfg.kappa, cfg.points, cfg.sigma, targets=tg, nthreads=NTHREADS)
    em = oracle.rel_l2(um[tg], u0)
    print(f"[gpu] {cfg.name} full n={cfg.n} mixed rel_l2={em:.3e}", flush=True)
    assert em <= 1e-6


# 3D Laplace M2L in mixed precision: FP32 contraction for P <= 16 when
# tol >= 1e-6 (P = 9 and 14 here with separation 2), FP64 otherwise (P = 17
# with separation 1); both against the oracle and the FP64 plan.
@pytest.mark.parametrize("tol,sep", [(1e-4, 2), (1e-6, 2), (1e-4, 1)])
def test_laplace_mixed_m2l(tol, sep):
    cfg = synth.make_config(2, n=44 * 44)
    u0 = oracle.direct_self(3, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    print(f"[gpu] laplace mixed m2l tol={tol} sep={sep}", flush=True)
    outs = {}
    for prec in ("mixed", "fp64"):
        plan = cf.Plan(torch.from_numpy(cfg.points).cuda(), "laplace", 0.0, tol, precision=prec, leaf_size=32,
                       separation=sep)
        u = plan(torch.from_numpy(cfg.sigma).cuda())
        torch.cuda.synchronize()
        outs[prec] = (u.cpu().numpy(), plan.info()["max_p"])
    em, ed = oracle.rel_l2(outs["mixed"][0], u0), oracle.rel_l2(outs["fp64"][0], u0)
    print(f"[gpu] P={outs['mixed'][1]}: mixed rel_l2={em:.3e}  fp64 rel_l2={ed:.3e}", flush=True)
    assert em <= tol
    # the mixed result stays within its rounding floor of the FP64 one
    assert oracle.rel_l2(outs["mixed"][0], outs["fp64"][0]) <= 1e-6
