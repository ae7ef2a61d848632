"""GPU parity of the 3D Helmholtz path (through the C-ABI) against the oracle."""
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
K3 = synth.KAPPA_C3


def _say(msg):
    print(msg, flush=True)


def _plan_eval(pts, sig, kappa, tol, leaf=0, sep=0):
    _say(f"[gpu] h3d plan n={pts.shape[0]} kappa={kappa:.4g} tol={tol} leaf={leaf} sep={sep}")
    plan = cf.Plan(torch.from_numpy(pts).cuda(), "helmholtz", kappa, tol, leaf_size=leaf, separation=sep)
    u = plan(torch.from_numpy(sig).cuda())
    torch.cuda.synchronize()
    return plan, u.cpu().numpy()


@pytest.mark.parametrize("m,tol,leaf", [(40, 1e-6, 64), (40, 1e-10, 64), (56, 1e-10, 32), (48, 1e-6, 16)])
def test_c3_family_full_parity(m, tol, leaf):
    cfg = synth.make_config(3, n=m * m)
    plan, u = _plan_eval(cfg.points, cfg.sigma, K3, tol, leaf)
    u0 = oracle.direct_self(3, "helmholtz", K3, cfg.points, cfg.sigma, nthreads=NTHREADS)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] h3d m={m} tol={tol} leaf={leaf} rel_l2={e:.3e} P={plan.nterms()} info={plan.info()}")
    assert e <= tol


@pytest.mark.parametrize("kappa", [0.5, 3.0, 25.0])
def test_wavenumber_range_parity(kappa):
    cfg = synth.make_config(3, n=40 * 40)
    pts = cfg.points * min(1.0, K3 / kappa)
    plan, u = _plan_eval(pts, cfg.sigma, kappa, 1e-8, 32)
    u0 = oracle.direct_self(3, "helmholtz", kappa, pts, cfg.sigma, nthreads=NTHREADS)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] h3d kappa={kappa} rel_l2={e:.3e} P={plan.nterms()}")
    assert e <= 1e-8


def test_tree_and_lists_bit_exact():
    cfg = synth.make_config(3, n=56 * 56)
    plan, _ = _plan_eval(cfg.points, cfg.sigma, K3, 1e-6, 24)
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
    rng = np.random.default_rng(91)
    a = rng.normal(0, 0.03, (1500, 3)) + 0.3
    b = rng.uniform(-1, 1, (1500, 3))
    re = np.concatenate([a, b])
    pts = re + 0.1j * np.abs(re)
    sig = synth.density(pts.shape[0], 92)
    plan, u = _plan_eval(pts, sig, 6.0, 1e-8, 16)
    info = plan.info()
    assert info["n_list3"] > 0 and info["n_list4"] > 0
    u0 = oracle.direct_self(3, "helmholtz", 6.0, pts, sig, nthreads=NTHREADS)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] h3d clustered rel_l2={e:.3e}")
    assert e <= 1e-8


def test_deterministic():
    cfg = synth.make_config(3, n=32 * 32)
    plan, u1 = _plan_eval(cfg.points, cfg.sigma, K3, 1e-8, 32)
    u2 = plan(cfg.sigma)
    assert np.array_equal(u1, u2)


def test_zz_c3_full_size_sampled_parity():
    cfg = synth.make_config(3, n_oracle=1024)
    plan, u = _plan_eval(cfg.points, cfg.sigma, K3, 1e-10)
    tg = cfg.oracle_targets
    u0 = oracle.direct_self(3, "helmholtz", K3, cfg.points, cfg.sigma, targets=tg, nthreads=NTHREADS)
    e = oracle.rel_l2(u[tg], u0)
    _say(f"[gpu] c3 full n={cfg.n} rel_l2={e:.3e} P={plan.nterms()} info={plan.info()}")
    assert e <= 1e-10
