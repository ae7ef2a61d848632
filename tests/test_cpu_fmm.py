"""The CPU FMM reference (the host-core baseline bench.py times beside the
GPU path) against the oracle's direct sum."""
import numpy as np
import pytest

import cpu_ref
import oracle
import synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    cpu_ref.build(force=False)


@pytest.mark.parametrize("m,tol,leaf", [(48, 1e-6, 256), (40, 1e-10, 64), (40, 1e-4, 32)])
def test_cpu_fmm_matches_oracle(m, tol, leaf):
    cfg = synth.make_config(2, n=m * m)
    u, (tp, te) = cpu_ref.fmm3d_laplace(cfg.points, cfg.sigma, tol, leaf_size=leaf, sep=2, nthreads=4)
    u0 = oracle.direct_self(3, "laplace", 0.0, cfg.points, cfg.sigma, nthreads=4)
    assert oracle.rel_l2(u, u0) <= tol
    assert tp >= 0.0 and te > 0.0


def test_cpu_fmm_clustered_tree():
    rng = np.random.default_rng(77)
    a = rng.normal(0, 0.03, (1500, 3)) + 0.3
    b = rng.uniform(-1, 1, (1500, 3))
    re = np.concatenate([a, b])
    pts = re + 0.1j * np.abs(re)
    sig = synth.density(pts.shape[0], 78)
    u, _ = cpu_ref.fmm3d_laplace(pts, sig, 1e-6, leaf_size=16, sep=2, nthreads=4)
    u0 = oracle.direct_self(3, "laplace", 0.0, pts, sig, nthreads=4)
    assert oracle.rel_l2(u, u0) <= 1e-6
