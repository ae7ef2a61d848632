"""GPU parity of the 2D Laplace path (Sec. 4.2; G = -(1/2 pi) log r) through
the C-ABI against the oracle's direct FP64 sum, and its integer tree against
the oracle tree."""
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


def _run(pts, sig, tol, leaf=0, sep=0, targets=None):
    _say(f"[gpu] l2d plan n={pts.shape[0]} tol={tol} leaf={leaf} sep={sep} "
         f"targets={None if targets is None else targets.shape[0]}")
    plan = cf.Plan(torch.from_numpy(pts).cuda(), "laplace", 0.0, tol, leaf_size=leaf, separation=sep,
                   targets=None if targets is None else torch.from_numpy(targets).cuda())
    u = plan(torch.from_numpy(sig).cuda())
    plan.sync()
    return plan, u.cpu().numpy()


@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-12])
def test_c0_curve_full_parity(tol):
    cfg = synth.make_config(0)
    plan, u = _run(cfg.points, cfg.sigma, tol)
    u0 = oracle.direct_self(2, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] l2d c0 tol={tol} rel_l2={e:.3e} P={plan.nterms()} info={plan.info()}")
    assert e <= tol


@pytest.mark.parametrize("n,tol", [(1 << 16, 1e-6), (1 << 16, 1e-12)])
def test_c1_curve_sampled_parity(n, tol):
    cfg = synth.make_config(1, n=n, n_oracle=512)
    plan, u = _run(cfg.points, cfg.sigma, tol)
    tg = cfg.oracle_targets
    u0 = oracle.direct_self(2, "laplace", 0.0, cfg.points, cfg.sigma, targets=tg, nthreads=NTHREADS)
    e = oracle.rel_l2(u[tg], u0)
    _say(f"[gpu] l2d c1 n={n} tol={tol} rel_l2={e:.3e} info={plan.info()}")
    assert e <= tol


def test_tree_bit_exact():
    cfg = synth.make_config(0)
    plan, _ = _run(cfg.points, cfg.sigma, 1e-8)
    info = plan.info()
    t = T.build_tree(cfg.points, info["leaf_size"], info["separation"], info["top_level"])
    ex = plan.export_tree()
    assert np.array_equal(ex["keys"], t.keys) and np.array_equal(ex["perm"], t.perm)
    for q in range(1, 5):
        off, idx = plan.export_list(q)
        assert np.array_equal(off, t.lists[f"L{q}"][0]) and np.array_equal(idx, t.lists[f"L{q}"][1])


@pytest.mark.parametrize("leaf,sep", [(8, 1), (17, 2), (200, 1), (64, 2)])
def test_leaf_sizes_and_separation(leaf, sep):
    cfg = synth.make_config(0, n=2500)
    plan, u = _run(cfg.points, cfg.sigma, 1e-9, leaf=leaf, sep=sep)
    u0 = oracle.direct_self(2, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] l2d leaf={leaf} sep={sep} rel_l2={e:.3e}")
    assert e <= 1e-9


def test_clustered_adaptive_tree_uses_lists_3_and_4():
    rng = np.random.default_rng(91)
    a = rng.normal(0, 0.01, (1500, 2)) + 0.3
    b = rng.uniform(-1, 1, (1500, 2))
    re = np.concatenate([a, b])
    pts = re + 0.2j * np.abs(re)
    sig = synth.density(pts.shape[0], 92)
    plan, u = _run(pts, sig, 1e-8, leaf=8)
    info = plan.info()
    assert info["n_list3"] > 0 and info["n_list4"] > 0
    u0 = oracle.direct_self(2, "laplace", 0.0, pts, sig, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-8


def test_real_coordinates_and_coincident_points():
    cfg = synth.make_config(0, n=3000)
    pts = cfg.points.real.astype(np.complex128)
    pts[100] = pts[7]                                  # a coincident pair contributes nothing
    plan, u = _run(pts, cfg.sigma, 1e-10)
    u0 = oracle.direct_self(2, "laplace", 0.0, pts, cfg.sigma, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-10


def test_distinct_targets():
    cfg = synth.make_config(0, n=3000)
    trg = synth.curve2d(1700, 9400)
    trg[:3] = cfg.points[[5, 50, 500]]
    plan, u = _run(cfg.points, cfg.sigma, 1e-10, targets=trg)
    u0 = oracle.direct(2, "laplace", 0.0, trg, cfg.points, cfg.sigma, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 3, 65, 129])
def test_tiny_inputs(n):
    cfg = synth.make_config(0, n=n)
    plan, u = _run(cfg.points, cfg.sigma, 1e-10)
    u0 = oracle.direct_self(2, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    if n == 1:
        assert np.all(u == 0)
    else:
        assert oracle.rel_l2(u, u0) <= 1e-12


def test_deterministic_and_host_path():
    cfg = synth.make_config(0, n=2000)
    plan, u1 = _run(cfg.points, cfg.sigma, 1e-8)
    u2 = plan(cfg.sigma)
    assert np.array_equal(u1, u2)
