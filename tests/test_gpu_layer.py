"""GPU parity of the 3D Laplace layer potentials (Sec. 2.1: single and double
layer, and the gradients behind the normal derivatives S', D') through the
C-ABI against the oracle's direct sums."""
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
# gradients are one derivative rougher than the potentials the expansion
# length is chosen for: their gate is GRAD_FACTOR x tol
GRAD_FACTOR = 10.0


def _say(msg):
    print(msg, flush=True)


def _normals(pts, seed):
    """Complex 'normals' of the plane family: unit-size complex vectors."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((pts.shape[0], 3)) + 0.3j * rng.standard_normal((pts.shape[0], 3))
    return v


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("m,tol,leaf", [(48, 1e-6, 0), (40, 1e-10, 64), (44, 1e-8, 32)])
def test_charges_and_dipoles_potential_and_gradient(m, tol, leaf):
    cfg = synth.make_config(2, n=m * m)
    pts = cfg.points
    q = cfg.sigma
    v = _normals(pts, 700 + m) * synth.density(pts.shape[0], 800 + m)[:, None]
    _say(f"[gpu] layer n={pts.shape[0]} tol={tol} leaf={leaf}")
    plan = cf.Plan(torch.from_numpy(pts).cuda(), "laplace", 0.0, tol, leaf_size=leaf)
    u, g = plan.eval_layer(torch.from_numpy(q).cuda(), torch.from_numpy(v).cuda(), gradient=True)
    plan.sync()
    u0, g0 = oracle.layer3_self("laplace", 0.0, pts, charge=q, dipole=v, nthreads=NTHREADS)
    eu, eg = _rel(u.cpu().numpy(), u0), _rel(g.cpu().numpy(), g0)
    _say(f"[gpu] layer n={pts.shape[0]} tol={tol} potential {eu:.3e} gradient {eg:.3e} info={plan.info()}")
    assert eu <= tol and eg <= GRAD_FACTOR * tol


def test_double_layer_alone_and_normal_derivative():
    cfg = synth.make_config(2, n=40 * 40)
    pts = cfg.points
    nu = _normals(pts, 9)
    tau = synth.density(pts.shape[0], 10)
    plan = cf.Plan(pts, "laplace", 0.0, 1e-8)
    u, g = plan.eval_layer(None, nu * tau[:, None], potential=True, gradient=True)
    u0, g0 = oracle.layer3_self("laplace", 0.0, pts, dipole=nu * tau[:, None], nthreads=NTHREADS)
    # D[tau] and D'[tau] = nu . grad D[tau]
    dp, dp0 = np.sum(nu * g, axis=1), np.sum(nu * g0, axis=1)
    eu, ed = _rel(u, u0), _rel(dp, dp0)
    _say(f"[gpu] double layer {eu:.3e}, D' {ed:.3e}")
    assert eu <= 1e-8 and ed <= GRAD_FACTOR * 1e-8
    # S' alone (gradient only, charges only)
    _, g = plan.eval_layer(cfg.sigma, None, potential=False, gradient=True)
    _, g0 = oracle.layer3_self("laplace", 0.0, pts, charge=cfg.sigma, nthreads=NTHREADS)
    sp, sp0 = np.sum(nu * g, axis=1), np.sum(nu * g0, axis=1)
    assert _rel(sp, sp0) <= GRAD_FACTOR * 1e-8
    # the charge-only potential of the layer path equals cfmm_eval's
    u1, _ = plan.eval_layer(cfg.sigma, None)
    assert _rel(u1, plan(cfg.sigma)) <= 1e-13


def test_clustered_tree_uses_dipole_p2l_and_gradient_m2p():
    rng = np.random.default_rng(77)
    a = rng.normal(0, 0.03, (1500, 3)) + 0.3
    b = rng.uniform(-1, 1, (1500, 3))
    re = np.concatenate([a, b])
    pts = re + 0.1j * np.abs(re)
    q = synth.density(pts.shape[0], 78)
    v = _normals(pts, 79)
    plan = cf.Plan(torch.from_numpy(pts).cuda(), "laplace", 0.0, 1e-8, leaf_size=16)
    info = plan.info()
    assert info["n_list3"] > 0 and info["n_list4"] > 0
    u, g = plan.eval_layer(torch.from_numpy(q).cuda(), torch.from_numpy(v).cuda(), gradient=True)
    plan.sync()
    u0, g0 = oracle.layer3_self("laplace", 0.0, pts, charge=q, dipole=v, nthreads=NTHREADS)
    eu, eg = _rel(u.cpu().numpy(), u0), _rel(g.cpu().numpy(), g0)
    _say(f"[gpu] layer clustered potential {eu:.3e} gradient {eg:.3e}")
    assert eu <= 1e-8 and eg <= GRAD_FACTOR * 1e-8


def test_distinct_targets_and_host_path():
    cfg = synth.make_config(2, n=36 * 36)
    src = cfg.points
    trg = synth.plane3d_grid(30, lo=-5.93, hi=5.97)
    trg[:2] = src[[3, 400]]
    v = _normals(src, 11)
    plan = cf.Plan(src, "laplace", 0.0, 1e-9, targets=trg)
    u, g = plan.eval_layer(cfg.sigma, v, gradient=True)
    u0, g0 = oracle.layer3("laplace", 0.0, trg, src, charge=cfg.sigma, dipole=v, nthreads=NTHREADS)
    eu, eg = _rel(u, u0), _rel(g, g0)
    _say(f"[gpu] layer targets potential {eu:.3e} gradient {eg:.3e}")
    assert eu <= 1e-9 and eg <= GRAD_FACTOR * 1e-9


def test_layer_not_supported_outside_3d_laplace():
    cfg = synth.make_config(0, n=500)
    plan = cf.Plan(cfg.points, "helmholtz", 10.0, 1e-6)
    with pytest.raises(cf.CfmmError) as ei:
        plan.eval_layer(cfg.sigma, None)
    assert ei.value.code == cf.CFMM_ENOTSUP
