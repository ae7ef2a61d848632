"""The device tree topology (Sec. 6.1: occupancy split, level restriction) and
Lists 1-4 (Sec. 6.2) bit for bit against the oracle's tree, over uniform,
clustered and sparse point sets in 2D and 3D, both separations, several leaf
sizes, and trees with leaves coarser than the far field's top level (such a
leaf is near every box)."""
import numpy as np
import pytest

import synth
from oracle import tree as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2509_05458_amd as cf  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _clustered(dim, n, seed, outliers=0):
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, 0.02, (n // 2, dim)) + 0.25
    b = rng.uniform(-1.0, 1.0, (n - n // 2, dim))
    re = np.concatenate([a, b])
    if outliers:
        far = rng.uniform(2.5, 3.0, (outliers, dim))
        re = np.concatenate([re, far])
    return re + 0.1j * np.abs(re)


def _cases():
    c0 = synth.make_config(0).points
    # (name, points, kernel, kappa, leaf size, separation, tol); the last two
    # start the far field below some leaves (the literal 2D curve and a 3D
    # plane many wavelengths across at a tight tolerance)
    return [
        ("2d-curve", c0, "helmholtz", 10.0, 16, 1, 1e-6),
        ("2d-curve-k2", c0, "helmholtz", 10.0, 9, 2, 1e-6),
        ("2d-clustered", _clustered(2, 6000, 11), "laplace", 0.0, 8, 1, 1e-6),
        ("2d-clustered-k2", _clustered(2, 6000, 12), "helmholtz", 30.0, 8, 2, 1e-6),
        ("2d-outliers", _clustered(2, 6000, 13, outliers=5), "helmholtz", 60.0, 8, 1, 1e-6),
        ("3d-plane", synth.plane3d_grid(48), "laplace", 0.0, 16, 2, 1e-6),
        ("3d-clustered", _clustered(3, 6000, 14), "helmholtz", 6.0, 16, 2, 1e-6),
        ("3d-clustered-k1", _clustered(3, 6000, 15), "laplace", 0.0, 12, 1, 1e-6),
        ("3d-outliers", _clustered(3, 6000, 16, outliers=7), "helmholtz", 20.0, 10, 2, 1e-6),
        ("2d-deep-top", synth.curve2d_literal(4096, 1301, 100.0), "helmholtz", 100.0, 64, 1, 1e-6),
        ("3d-deep-top", synth.plane3d_bumps(100, 1250), "helmholtz", 26.18, 16, 2, 1e-10),
    ]


CASES = _cases()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_device_tree_and_lists_bit_exact(case):
    name, pts, kernel, kappa, leaf, sep, tol = CASES[case]
    _say(f"[gpu] tree {name} n={pts.shape[0]} {kernel} kappa={kappa} leaf={leaf} sep={sep} tol={tol}")
    plan = cf.Plan(torch.from_numpy(pts).cuda(), kernel, kappa, tol, leaf_size=leaf, separation=sep)
    info = plan.info()
    t = T.build_tree(pts, leaf, sep, info["top_level"])
    ex = plan.export_tree()
    assert np.array_equal(ex["keys"], t.keys) and np.array_equal(ex["perm"], t.perm)
    for k in ("level", "parent", "child0", "nchild", "pbeg", "pend", "prefix"):
        assert np.array_equal(ex[k], getattr(t, k).astype(ex[k].dtype)), k
    for q in range(1, 5):
        off, idx = plan.export_list(q)
        assert np.array_equal(off, t.lists[f"L{q}"][0]), f"L{q} offsets"
        assert np.array_equal(idx, t.lists[f"L{q}"][1]), f"L{q} entries"
    coarse = int(np.sum((ex["nchild"] == 0) & (ex["level"] < info["top_level"])))
    _say(f"[gpu] tree {name} ok: nbox={info['nbox']} top={info['top_level']} coarse_leaves={coarse} "
         f"timing={plan.timing()}")


def test_some_case_has_leaves_coarser_than_top():
    found = False
    for name, pts, kernel, kappa, leaf, sep, tol in CASES:
        plan = cf.Plan(torch.from_numpy(pts).cuda(), kernel, kappa, tol, leaf_size=leaf, separation=sep)
        info = plan.info()
        ex = plan.export_tree()
        if np.any((ex["nchild"] == 0) & (ex["level"] < info["top_level"])):
            found = True
            break
    assert found


def test_plan_timing_phases():
    cfg = synth.make_config(0)
    plan = cf.Plan(torch.from_numpy(cfg.points).cuda(), "helmholtz", cfg.kappa, 1e-10)
    tm = plan.timing()
    parts = sum(tm[k] for k in ("keys_sort", "topology", "centres_p", "lists", "tables", "check"))
    assert all(v >= 0.0 for v in tm.values())
    assert abs(parts - tm["total"]) <= 1e-6 * max(1.0, tm["total"])
