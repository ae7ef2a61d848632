"""GPU checks of the GMRES driver on the library: second-kind systems
a sigma + S[w sigma] = f on a complexified curve (2D Helmholtz and Laplace)
and plane (3D Laplace), solved with one plan and many cfmm_eval matvecs; the
solution's residual is measured with the oracle's direct sum."""
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
from paper_2509_05458_amd import gmres as G  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


@pytest.mark.parametrize("dim,kernel,kappa,shift", [(2, "helmholtz", 4.0, 1.0), (2, "laplace", 0.0, 0.5),
                                                    (3, "laplace", 0.0, 0.5)])
def test_gmres_second_kind_solve(dim, kernel, kappa, shift):
    if dim == 2:
        pts, w = G.curve_nodes(3000)
    else:
        m = 40
        pts = synth.plane3d_grid(m)
        w = np.full(pts.shape[0], (12.0 / (m - 1)) ** 2, dtype=np.complex128)
    f = synth.density(pts.shape[0], 555)
    print(f"[gpu] gmres {dim}D {kernel} n={pts.shape[0]}", flush=True)
    plan = cf.Plan(torch.from_numpy(pts).cuda(), kernel, kappa, 1e-10)
    wt = torch.from_numpy(w).cuda()
    op = G.LayerOperator(plan, wt, shift)
    x, info = G.gmres(op, torch.from_numpy(f).cuda(), tol=1e-7, restart=60, maxiter=600)
    plan.sync()
    assert info.converged, info.residuals[-5:]
    assert op.calls >= info.iterations
    xs = x.cpu().numpy()
    # true residual with the oracle's direct sum
    u0 = oracle.direct_self(dim, kernel, kappa, pts, w * xs, nthreads=NTHREADS)
    res = np.linalg.norm(shift * xs + u0 - f) / np.linalg.norm(f)
    print(f"[gpu] gmres {dim}D {kernel}: {info.iterations} matvecs, residual {res:.2e}", flush=True)
    assert res <= 1e-6
