"""GPU parity of the 2D Helmholtz path (through the C-ABI) against the oracle:
the direct FP64 sum for the potentials, the oracle tree for the integer work."""
import dataclasses
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


def _oracle(cfg, targets):
    return oracle.direct_self(2, "helmholtz", cfg.kappa, cfg.points, cfg.sigma,
                              targets=targets, nthreads=NTHREADS)


def _run(cfg, tol, leaf=0, sep=0, device=True):
    _say(f"[gpu] plan {cfg.name} n={cfg.n} tol={tol} leaf={leaf} sep={sep}")
    if device:
        pts = torch.from_numpy(cfg.points).cuda()
        plan = cf.Plan(pts, "helmholtz", cfg.kappa, tol, leaf_size=leaf, separation=sep)
        u = plan(torch.from_numpy(cfg.sigma).cuda())
        torch.cuda.synchronize()
        return plan, u.cpu().numpy()
    plan = cf.Plan(cfg.points, "helmholtz", cfg.kappa, tol, leaf_size=leaf, separation=sep)
    return plan, plan(cfg.sigma)


@pytest.mark.parametrize("tol", [1e-10, 1e-6])
def test_c0_full_parity(tol):
    cfg = synth.make_config(0)
    plan, u = _run(cfg, tol)
    u0 = _oracle(cfg, None)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] c0 tol={tol} rel_l2={e:.3e} info={plan.info()}")
    assert e <= tol


def test_c0_tree_bit_exact_and_centres():
    cfg = synth.make_config(0)
    plan, _ = _run(cfg, 1e-10)
    info = plan.info()
    t = T.build_tree(cfg.points, info["leaf_size"], info["separation"], info["top_level"])
    ex = plan.export_tree()
    assert np.array_equal(ex["keys"], t.keys)
    assert np.array_equal(ex["perm"], t.perm)
    for k in ("level", "parent", "child0", "nchild", "pbeg", "pend", "prefix"):
        assert np.array_equal(ex[k], getattr(t, k).astype(ex[k].dtype)), k
    for q in range(1, 5):
        off, idx = plan.export_list(q)
        assert np.array_equal(off, t.lists[f"L{q}"][0]) and np.array_equal(idx, t.lists[f"L{q}"][1])
    cen = plan.export_centers()
    ref = T.complex_centers(t, cfg.points)
    assert np.array_equal(cen.real, ref.real)
    assert np.max(np.abs(cen.imag - ref.imag)) <= 1e-14 * max(1.0, np.max(np.abs(ref.imag)))


@pytest.mark.parametrize("n,tol", [(1 << 16, 1e-6), (1 << 16, 1e-12), (20000, 1e-10)])
def test_c1_family_sampled_parity(n, tol):
    cfg = synth.make_config(1, n=n, n_oracle=512)
    plan, u = _run(cfg, tol)
    tg = cfg.oracle_targets
    u0 = _oracle(cfg, tg)
    e = oracle.rel_l2(u[tg], u0)
    _say(f"[gpu] c1 n={n} tol={tol} rel_l2={e:.3e} info={plan.info()}")
    assert e <= tol


@pytest.mark.parametrize("tol", [1e-6, 1e-12])
def test_c1_full_size_sampled_parity(tol):
    cfg = synth.make_config(1, n_oracle=256)
    plan, u = _run(cfg, tol)
    tg = cfg.oracle_targets
    u0 = _oracle(cfg, tg)
    e = oracle.rel_l2(u[tg], u0)
    _say(f"[gpu] c1 full n={cfg.n} tol={tol} rel_l2={e:.3e} info={plan.info()}")
    assert e <= tol
    t = plan.export_tree()
    # the permutation is a permutation and keys are sorted (the tree is checked
    # bit for bit against the oracle at smaller sizes)
    assert np.array_equal(np.sort(t["perm"]), np.arange(cfg.n))
    assert np.all(t["keys"][1:] >= t["keys"][:-1])


def test_c1_tree_bit_exact_at_64k():
    cfg = synth.make_config(1, n=1 << 16)
    plan, _ = _run(cfg, 1e-6)
    info = plan.info()
    t = T.build_tree(cfg.points, info["leaf_size"], info["separation"], info["top_level"])
    ex = plan.export_tree()
    assert np.array_equal(ex["keys"], t.keys) and np.array_equal(ex["perm"], t.perm)
    for q in range(1, 5):
        off, idx = plan.export_list(q)
        assert np.array_equal(idx, t.lists[f"L{q}"][1])


def test_deterministic_and_host_device_paths_agree():
    cfg = synth.make_config(0, n=3000)
    plan, u1 = _run(cfg, 1e-8)
    u2 = plan(torch.from_numpy(cfg.sigma).cuda()).cpu().numpy()
    assert np.array_equal(u1, u2)
    u3 = plan(cfg.sigma)
    assert np.array_equal(u1, u3)


@pytest.mark.parametrize("leaf,sep", [(8, 1), (17, 2), (200, 1)])
def test_leaf_sizes_and_separation(leaf, sep):
    cfg = synth.make_config(0, n=2500)
    plan, u = _run(cfg, 1e-9, leaf=leaf, sep=sep)
    u0 = _oracle(cfg, None)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] leaf={leaf} sep={sep} rel_l2={e:.3e}")
    assert e <= 1e-9


@pytest.mark.parametrize("n", [1, 2, 3, 65, 129])
def test_tiny_inputs(n):
    cfg = synth.make_config(0, n=n)
    plan, u = _run(cfg, 1e-10)
    u0 = _oracle(cfg, None)
    if n == 1:
        assert np.all(u == 0)
    else:
        assert oracle.rel_l2(u, u0) <= 1e-12


def test_real_coordinates_and_coincident_points():
    """Im = 0 reduces to the textbook kernel; an exact duplicate point
    contributes nothing to its twin (a pair at s = 0)."""
    cfg = synth.make_config(0, n=3000)
    pts = cfg.points.real.astype(np.complex128)
    pts[100] = pts[7]
    c2 = dataclasses.replace(cfg, points=pts)
    plan, u = _run(c2, 1e-10)
    u0 = _oracle(c2, None)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] h2d real+coincident rel_l2={e:.3e}")
    assert e <= 1e-10


def test_invalid_geometry_is_rejected():
    pts = np.array([[0.0, 0.0], [1.0, 1.2j]], dtype=np.complex128)
    with pytest.raises(cf.CfmmError) as ei:
        cf.Plan(pts, "helmholtz", 1.0, 1e-6)
    assert ei.value.code == cf.CFMM_EGEOMETRY
    bad = np.array([[0.0, 0.0], [np.nan, 0.0]], dtype=np.complex128)
    with pytest.raises(cf.CfmmError) as ei:
        cf.Plan(bad, "helmholtz", 1.0, 1e-6)
    assert ei.value.code == cf.CFMM_EGEOMETRY


def test_profiling_modes():
    """Mode 1 brackets every stage of the last evaluation; mode 2 keeps the
    near-field time of back-to-back evaluations (ring of 64) without a host
    sync between them; other modes are rejected."""
    cfg = synth.make_config(0)
    pts = torch.from_numpy(cfg.points).cuda()
    sig = torch.from_numpy(cfg.sigma).cuda()
    plan = cf.Plan(pts, "helmholtz", cfg.kappa, 1e-6)
    out = torch.empty_like(sig)
    plan.set_profiling(1)
    plan.eval_into(sig, out)
    torch.cuda.synchronize()
    st = plan.stage_ms()
    assert all(v >= 0.0 for v in st.values()) and st["eval"] > 0.0
    plan.set_profiling(2)
    for _ in range(3):
        plan.eval_into(sig, out)
    torch.cuda.synchronize()
    tot, cnt = plan.ring_ms()
    assert cnt == 3 and tot > 0.0
    for _ in range(70):
        plan.eval_into(sig, out)
    torch.cuda.synchronize()
    tot2, cnt2 = plan.ring_ms()
    assert cnt2 == 64 and tot2 > 0.0
    plan.set_profiling(3)
    for _ in range(2):
        plan.eval_into(sig, out)
    torch.cuda.synchronize()
    tot3, cnt3 = plan.ring_ms()
    assert cnt3 == 2 and 0.0 < tot3 < 2 * st["eval"] + 1.0
    plan.set_profiling(0)
    with pytest.raises(cf.CfmmError):
        plan.set_profiling(4)
    u0 = plan(sig).cpu().numpy()
    assert oracle.rel_l2(u0, out.cpu().numpy()) == 0.0


@pytest.mark.parametrize("leaf,kappa", [(8, 100.0), (24, 100.0), (128, 15.0)])
def test_series_pair_walk_leaf_sizes(leaf, kappa):
    """The small-argument near field of the C1 curve (scale 0.1) at leaf
    sizes whose tiles need several slot passes per step (8, 24) or several
    tiles per leaf (128; kappa lowered so that those boxes stay in the series
    regime); every potential against the direct sum."""
    cfg = dataclasses.replace(synth.make_config(1, n=6000), kappa=kappa)
    plan, u = _run(cfg, 1e-9, leaf=leaf)
    nw = plan.near_work()
    assert nw["evaluations"] < nw["interactions"]     # symmetric items ran
    u0 = _oracle(cfg, None)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] c1 n=6000 leaf={leaf} rel_l2={e:.3e} near={nw}")
    assert e <= 1e-9
