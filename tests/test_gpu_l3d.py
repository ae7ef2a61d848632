"""GPU parity of the 3D Laplace path (through the C-ABI) against the oracle."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import tree as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2509_05458_amd as cf  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def _say(msg):
    print(msg, flush=True)


def _plan_eval(pts, sig, tol, leaf=0, sep=0):
    _say(f"[gpu] l3d plan n={pts.shape[0]} tol={tol} leaf={leaf} sep={sep}")
    plan = cf.Plan(torch.from_numpy(pts).cuda(), "laplace", 0.0, tol, leaf_size=leaf, separation=sep)
    u = plan(torch.from_numpy(sig).cuda())
    torch.cuda.synchronize()
    return plan, u.cpu().numpy()


# The expansion lengths span every M2L register-block count: P = 9, 14, 20,
# 22, 27, 31 with separation 2 and P = 17, 26 with separation 1 hold 1..5
# groups of four outputs per lane.  With separation 1 the plane's imaginary
# parts are scaled by `im` (Lipschitz constant 0.5 im): at the full 0.5 the
# k = 1 lists lie outside the proven 3D convergence region and the error
# stalls near 1e-4 at tol 1e-6.
@pytest.mark.parametrize("m,tol,leaf,sep,im", [
    (48, 1e-6, 32, 0, 1.0), (64, 1e-6, 64, 0, 1.0), (64, 1e-9, 64, 0, 1.0), (40, 1e-6, 256, 0, 1.0),
    (48, 1e-4, 16, 0, 1.0), (40, 1e-10, 64, 2, 1.0), (40, 1e-12, 64, 2, 1.0), (32, 1e-12, 32, 2, 1.0),
    (40, 1e-4, 32, 1, 1.0), (32, 1e-6, 32, 1, 0.2)])
def test_c2_family_full_parity(m, tol, leaf, sep, im):
    cfg = synth.make_config(2, n=m * m)
    pts = cfg.points.real + 1j * im * cfg.points.imag
    plan, u = _plan_eval(pts, cfg.sigma, tol, leaf, sep)
    u0 = oracle.direct_self(3, "laplace", 0.0, pts, cfg.sigma, nthreads=NTHREADS)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] l3d m={m} tol={tol} sep={sep} im={im} rel_l2={e:.3e} info={plan.info()}")
    assert e <= tol


def test_c3_geometry_laplace_parity_and_tree():
    cfg = synth.make_config(3, n=56 * 56)
    plan, u = _plan_eval(cfg.points, cfg.sigma, 1e-6, 24)
    u0 = oracle.direct_self(3, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-6
    info = plan.info()
    t = T.build_tree(cfg.points, info["leaf_size"], info["separation"], info["top_level"])
    ex = plan.export_tree()
    assert np.array_equal(ex["keys"], t.keys) and np.array_equal(ex["perm"], t.perm)
    for k in ("level", "parent", "child0", "nchild", "pbeg", "pend", "prefix"):
        assert np.array_equal(ex[k], getattr(t, k).astype(ex[k].dtype)), k
    for q in range(1, 5):
        off, idx = plan.export_list(q)
        assert np.array_equal(off, t.lists[f"L{q}"][0]) and np.array_equal(idx, t.lists[f"L{q}"][1])


def test_clustered_adaptive_tree_parity():
    rng = np.random.default_rng(77)
    a = rng.normal(0, 0.03, (1500, 3)) + 0.3
    b = rng.uniform(-1, 1, (1500, 3))
    re = np.concatenate([a, b])
    pts = re + 0.1j * np.abs(re)
    sig = synth.density(pts.shape[0], 78)
    plan, u = _plan_eval(pts, sig, 1e-6, 16)
    info = plan.info()
    assert info["n_list3"] > 0 and info["n_list4"] > 0
    u0 = oracle.direct_self(3, "laplace", 0.0, pts, sig, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-6


def test_c2_full_size_sampled_parity():
    # the configuration's 4096 seeded oracle targets
    cfg = synth.make_config(2, n_oracle=4096)
    plan, u = _plan_eval(cfg.points, cfg.sigma, 1e-6)
    tg = cfg.oracle_targets
    u0 = oracle.direct_self(3, "laplace", 0.0, cfg.points, cfg.sigma, targets=tg, nthreads=NTHREADS)
    e = oracle.rel_l2(u[tg], u0)
    _say(f"[gpu] c2 full n={cfg.n} rel_l2={e:.3e} info={plan.info()}")
    assert e <= 1e-6


def test_deterministic():
    cfg = synth.make_config(2, n=32 * 32)
    plan, u1 = _plan_eval(cfg.points, cfg.sigma, 1e-6, 32)
    u2 = plan(cfg.sigma)
    assert np.array_equal(u1, u2)
