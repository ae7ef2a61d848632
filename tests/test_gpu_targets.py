"""GPU parity with targets distinct from the sources (Sec. 2.3: targets x_i,
sources y_j), through the C-ABI, against the oracle's direct sum.  Targets lie
on the sources' surface (so the Lipschitz condition holds for every pair), a
few of them exactly on sources (a pair at squared distance 0 contributes
nothing), and their number differs from the sources'."""
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


def _targets(kind, n_src_pts, nt, seed):
    if kind == "h2d":
        t = synth.curve2d(nt, seed)
    elif kind == "l3d":
        m = int(round(np.sqrt(nt)))
        t = synth.plane3d_grid(m, lo=-5.93, hi=5.97)
    else:
        m = int(round(np.sqrt(nt)))
        t = synth.plane3d_bumps(m, synth.GEOM_SEED + 3, lo=-5.91, hi=5.95)
    # a few targets sit exactly on sources
    rng = np.random.default_rng(seed + 1)
    k = min(5, t.shape[0])
    t[:k] = n_src_pts[rng.choice(n_src_pts.shape[0], size=k, replace=False)]
    return t


CASES = [
    # kind, config, n_src, n_trg, kernel, kappa, tol
    ("h2d", 0, 3000, 2000, "helmholtz", 10.0, 1e-10),
    ("h2d", 0, 1500, 4500, "helmholtz", 10.0, 1e-6),
    ("l3d", 2, 48 * 48, 40 * 40, "laplace", 0.0, 1e-6),
    ("l3d", 2, 40 * 40, 56 * 56, "laplace", 0.0, 1e-10),
    ("h3d", 3, 44 * 44, 36 * 36, "helmholtz", synth.KAPPA_C3, 1e-10),
    ("h3d", 3, 36 * 36, 44 * 44, "helmholtz", synth.KAPPA_C3, 1e-6),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[2]}x{c[3]}-{c[6]:g}" for c in CASES])
def test_distinct_targets_parity(case):
    kind, ci, ns, nt, kern, kappa, tol = case
    cfg = synth.make_config(ci, n=ns)
    src, sig = cfg.points, cfg.sigma
    trg = _targets(kind, src, nt, 9100 + ci)
    _say(f"[gpu] targets {kind} n_src={src.shape[0]} n_trg={trg.shape[0]} tol={tol}")
    plan = cf.Plan(torch.from_numpy(src).cuda(), kern, kappa, tol,
                   targets=torch.from_numpy(trg).cuda())
    u = plan(torch.from_numpy(sig).cuda())
    plan.sync()
    u = u.cpu().numpy()
    info = plan.info()
    assert info["n_src"] == src.shape[0] and info["n_trg"] == trg.shape[0]
    assert info["n_points"] == src.shape[0] + trg.shape[0]
    u0 = oracle.direct(cfg.dim, kern, kappa, trg, src, sig, nthreads=NTHREADS)
    e = oracle.rel_l2(u, u0)
    _say(f"[gpu] targets {kind} rel_l2={e:.3e} info={info}")
    assert e <= tol


def test_distinct_targets_host_path_and_single_target():
    cfg = synth.make_config(0, n=2000)
    trg = synth.curve2d(1, 9200)
    plan = cf.Plan(cfg.points, "helmholtz", 10.0, 1e-10, targets=trg)
    u = plan(cfg.sigma)
    assert u.shape == (1,)
    u0 = oracle.direct(2, "helmholtz", 10.0, trg, cfg.points, cfg.sigma, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-10


def test_targets_equal_to_sources_match_the_self_plan_off_the_diagonal():
    """With targets = a copy of the sources, each target also meets its own
    source at distance 0 (contributing nothing), so the result equals the
    self-excluding plan's."""
    cfg = synth.make_config(2, n=32 * 32)
    a = cf.Plan(cfg.points, "laplace", 0.0, 1e-10)
    b = cf.Plan(cfg.points, "laplace", 0.0, 1e-10, targets=cfg.points.copy())
    ua, ub = a(cfg.sigma), b(cfg.sigma)
    u0 = oracle.direct_self(3, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=NTHREADS)
    assert oracle.rel_l2(ua, u0) <= 1e-10 and oracle.rel_l2(ub, u0) <= 1e-10


@pytest.mark.parametrize("kind,ci,kern,kappa", [("h2d", 0, "helmholtz", 10.0), ("l3d", 2, "laplace", 0.0),
                                               ("h3d", 3, "helmholtz", synth.KAPPA_C3)])
def test_non_finite_density_is_reported(kind, ci, kern, kappa):
    """A NaN density makes non-finite potentials: the host path returns
    CFMM_ERANGE, the device path reports it at the next sync, and the flag
    clears once reported."""
    cfg = synth.make_config(ci, n=1024 if ci else 1500)
    sig = cfg.sigma.copy()
    sig[7] = np.nan
    plan = cf.Plan(cfg.points, kern, kappa, 1e-6)
    with pytest.raises(cf.CfmmError) as ei:
        plan(sig)
    assert ei.value.code == cf.CFMM_ERANGE
    plan.sync()                                   # cleared
    u = plan(torch.from_numpy(sig).cuda())
    with pytest.raises(cf.CfmmError) as ei:
        plan.sync()
    assert ei.value.code == cf.CFMM_ERANGE
    assert not np.all(np.isfinite(u.cpu().numpy()))
    good = plan(cfg.sigma)                        # a finite density passes again
    assert np.all(np.isfinite(good))
