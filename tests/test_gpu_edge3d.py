"""3D edge cases through the C-ABI, against the oracle: tiny and ragged
inputs (single point, partial tiles, a single leaf), real coordinates (the
classical kernels), coincident points (a pair with r^2 = 0 contributes 0) and
rejected geometry (a near pair with Re r^2 <= 0)."""
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
KERNELS = [("laplace", 0.0), ("helmholtz", 3.0)]


def _points(n, seed, im=0.2):
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, (n, 3))
    return re + 1j * im * np.tanh(re)          # Lipschitz constant <= im


def _eval(pts, sig, kernel, kappa, tol, precision="fp64", leaf=0):
    print(f"[gpu] edge3d n={pts.shape[0]} {kernel} tol={tol} {precision} leaf={leaf}", flush=True)
    plan = cf.Plan(torch.from_numpy(pts).cuda(), kernel, kappa, tol, precision=precision, leaf_size=leaf)
    u = plan(torch.from_numpy(sig).cuda())
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("kernel,kappa", KERNELS)
@pytest.mark.parametrize("n", [1, 2, 3, 63, 65, 257, 1000])
def test_tiny_and_ragged(kernel, kappa, n):
    pts = _points(n, 100 + n)
    sig = synth.density(n, 200 + n)
    u = _eval(pts, sig, kernel, kappa, 1e-10, leaf=32)
    if n == 1:
        assert np.all(u == 0)
        return
    u0 = oracle.direct_self(3, kernel, kappa, pts, sig, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-10


@pytest.mark.parametrize("kernel,kappa", KERNELS)
def test_real_coordinates_reduce_to_classical(kernel, kappa):
    pts = _points(4000, 7, im=0.0)
    sig = synth.density(4000, 8)
    u = _eval(pts, sig, kernel, kappa, 1e-8, leaf=64)
    u0 = oracle.direct_self(3, kernel, kappa, pts, sig, nthreads=NTHREADS)
    assert oracle.rel_l2(u, u0) <= 1e-8


@pytest.mark.parametrize("kernel,kappa", KERNELS)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coincident_points_contribute_nothing(kernel, kappa, precision):
    pts = _points(1500, 9)
    pts[700] = pts[300]                        # two points at the same place
    sig = synth.density(1500, 10)
    tol = 1e-6
    u = _eval(pts, sig, kernel, kappa, tol, precision=precision, leaf=32)
    u0 = oracle.direct_self(3, kernel, kappa, pts, sig, nthreads=NTHREADS)
    assert np.all(np.isfinite(u))
    assert oracle.rel_l2(u, u0) <= tol


@pytest.mark.parametrize("kernel,kappa", KERNELS)
def test_invalid_geometry_is_rejected(kernel, kappa):
    # Re(r^2) = 1 - 1.44 < 0 for the two points, which are near each other
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.2j, 0.0]], dtype=np.complex128)
    with pytest.raises(cf.CfmmError) as ei:
        cf.Plan(pts, kernel, kappa, 1e-6)
    assert ei.value.code == cf.CFMM_EGEOMETRY
