"""3D Laplace M2L by point and shoot (Sec. 5.2: rotate the multipole so the
offset lies on the z axis, shift along it, rotate the local back) through the
C-ABI: the same evaluation with every pair in the direct addition-theorem
form (m2l_form "direct") and the oracle's direct sum.  The two forms compute
the same translation, so their results agree to rounding; geometries whose
offsets include near-null horizontal parts (x^2 + y^2 close to 0 at complex
points) keep those pairs in the direct form, and both forms then meet in one
evaluation."""
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


def _say(msg):
    print(msg, flush=True)


def _both(pts, sig, tol, leaf=0, precision="fp64"):
    out = {}
    for form in ("auto", "direct"):
        _say(f"[gpu] l3d pns n={pts.shape[0]} tol={tol} leaf={leaf} precision={precision} form={form}")
        plan = cf.Plan(torch.from_numpy(pts).cuda(), "laplace", 0.0, tol, leaf_size=leaf, precision=precision,
                       m2l_form=form)
        u = plan(torch.from_numpy(sig).cuda())
        torch.cuda.synchronize()
        out[form] = (plan, u.cpu().numpy())
    return out


def _vertical_mix(n, seed):
    # points in a cube whose imaginary parts turn with height, so that some
    # offsets of vertically stacked boxes have x^2 + y^2 near 0
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, (n, 3))
    im = np.stack([0.15 * np.sin(3.0 * re[:, 2]), 0.15 * np.cos(3.0 * re[:, 2]), 0.1 * re[:, 0]], axis=1)
    return re + 1j * im


# P = 14 (tol 1e-6), 9 (1e-4), 11 (1e-5) and 15 (2e-7: the largest length of
# the point-and-shoot lane layout, three wavefronts)
@pytest.mark.parametrize("m,tol,leaf", [(48, 1e-6, 32), (64, 1e-6, 64), (48, 1e-4, 16), (40, 1e-5, 24),
                                        (48, 2e-7, 32)])
def test_plane_pns_matches_direct_and_oracle(m, tol, leaf):
    cfg = synth.make_config(2, n=m * m)
    r = _both(cfg.points, cfg.sigma, tol, leaf)
    (pa, ua), (pd, ud) = r["auto"], r["direct"]
    wa, wd = pa.m2l_work(), pd.m2l_work()
    _say(f"[gpu] pns work auto={wa} direct={wd} P={pa.info()['max_p']}")
    if tol == 2e-7:
        assert pa.info()["max_p"] == 15
    assert wa["pns_pairs"] > 0 and wd["pns_pairs"] == 0
    assert wa["pns_pairs"] + wa["direct_pairs"] == wd["direct_pairs"] == pa.info()["n_list2"]
    d = oracle.rel_l2(ua, ud)
    u0 = oracle.direct_self(3, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    e = oracle.rel_l2(ua, u0)
    _say(f"[gpu] pns m={m} tol={tol} auto-vs-direct={d:.3e} rel_l2={e:.3e}")
    assert d <= 1e-11
    assert e <= tol


def test_both_forms_in_one_evaluation():
    pts = _vertical_mix(6000, 901)
    sig = synth.density(pts.shape[0], 902)
    r = _both(pts, sig, 1e-6, 32)
    (pa, ua), (pd, ud) = r["auto"], r["direct"]
    wa = pa.m2l_work()
    _say(f"[gpu] pns mixed forms work={wa}")
    assert wa["pns_pairs"] > 0 and wa["direct_pairs"] > 0
    u0 = oracle.direct_self(3, "laplace", 0.0, pts, sig, nthreads=NTHREADS)
    e, d = oracle.rel_l2(ua, u0), oracle.rel_l2(ua, ud)
    _say(f"[gpu] pns mixed forms rel_l2={e:.3e} auto-vs-direct={d:.3e}")
    assert d <= 1e-11
    assert e <= 1e-6


def test_mixed_precision_with_pns():
    cfg = synth.make_config(2, n=48 * 48)
    r = _both(cfg.points, cfg.sigma, 1e-6, 32, precision="mixed")
    pa, ua = r["auto"]
    assert pa.m2l_work()["pns_pairs"] > 0
    u0 = oracle.direct_self(3, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    e = oracle.rel_l2(ua, u0)
    _say(f"[gpu] pns mixed precision rel_l2={e:.3e}")
    assert e <= 1e-6


def test_out_of_range_lengths_use_the_direct_form():
    # P = 16 at tol 1e-7 (beyond the point-and-shoot lane layout) and tol
    # 1e-11: every pair stays in the direct form
    cfg = synth.make_config(2, n=32 * 32)
    for tol in (1e-7, 1e-11):
        plan = cf.Plan(torch.from_numpy(cfg.points).cuda(), "laplace", 0.0, tol, leaf_size=32)
        w = plan.m2l_work()
        _say(f"[gpu] pns off tol={tol} P={plan.info()['max_p']} work={w}")
        assert w["pns_pairs"] == 0 and w["direct_pairs"] == plan.info()["n_list2"]


def test_layer_potentials_with_pns():
    cfg = synth.make_config(2, n=40 * 40)
    pts = cfg.points
    n = pts.shape[0]
    rng = np.random.default_rng(903)
    v = (rng.standard_normal((n, 3)) + 0.3j * rng.standard_normal((n, 3))) * synth.density(n, 904)[:, None]
    q = synth.density(n, 905)
    res = {}
    for form in ("auto", "direct"):
        plan = cf.Plan(torch.from_numpy(pts).cuda(), "laplace", 0.0, 1e-6, leaf_size=32, m2l_form=form)
        u, g = plan.eval_layer(torch.from_numpy(q).cuda(), torch.from_numpy(v).cuda(), gradient=True)
        plan.sync()
        res[form] = (u.cpu().numpy(), g.cpu().numpy())
    assert oracle.rel_l2(res["auto"][0], res["direct"][0]) <= 1e-11
    assert oracle.rel_l2(res["auto"][1].ravel(), res["direct"][1].ravel()) <= 1e-10
