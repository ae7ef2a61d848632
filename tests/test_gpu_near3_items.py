"""3D near field with large leaves (256-point leaf size), through the C-ABI,
against the oracle's direct sum: leaves of 100 to 200 points take the
near-field items' full rows of 64 targets, partial rows, and a remainder of
at most 64 targets run with the roles swapped; a cluster of 70 coincident
points spans two 64-point tiles of one leaf, so the diagonal item's pair of
distinct tiles meets pairs with r^2 = 0 (which contribute 0)."""
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
KERNELS = [("laplace", 0.0), ("helmholtz", 2.0)]
N = 9600
LEAF = 256


def _points(seed, im=0.2):
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, (N, 3))
    return re + 1j * im * np.tanh(re)          # Lipschitz constant <= im


def _leaf_sizes(pts):
    t = T.build_tree(pts, LEAF, 2, 2)
    leaf = t.nchild == 0
    return (t.pend - t.pbeg)[leaf]


def _eval(pts, sig, kernel, kappa, tol, precision):
    print(f"[gpu] near3 items n={pts.shape[0]} {kernel} tol={tol} {precision} leaf={LEAF}", flush=True)
    plan = cf.Plan(torch.from_numpy(pts).cuda(), kernel, kappa, tol, precision=precision, leaf_size=LEAF)
    u = plan(torch.from_numpy(sig).cuda())
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("kernel,kappa", KERNELS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_large_leaves(kernel, kappa, precision, tol):
    pts = _points(31)
    sizes = _leaf_sizes(pts)
    # the shapes the items are cut into: leaves above 128 points with a
    # remainder of at most 64, and leaves below 128
    assert np.any((sizes > 128) & (sizes <= 192)) and np.any(sizes < 128), np.unique(sizes)
    sig = synth.density(N, 32)
    u = _eval(pts, sig, kernel, kappa, tol, precision)
    u0 = oracle.direct_self(3, kernel, kappa, pts, sig, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= tol


@pytest.mark.parametrize("kernel,kappa", KERNELS)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_coincident_cluster_across_tiles(kernel, kappa, precision, tol):
    pts = _points(33)
    pts[1:70] = pts[0]                          # 70 points at one place, one Morton key
    sizes = _leaf_sizes(pts)
    assert sizes.max() > 70
    sig = synth.density(N, 34)
    u = _eval(pts, sig, kernel, kappa, tol, precision)
    assert np.all(np.isfinite(u))
    u0 = oracle.direct_self(3, kernel, kappa, pts, sig, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= tol
