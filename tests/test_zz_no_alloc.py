"""cfmm_eval_static, the evaluation entry point for callers that cannot
allocate, through the C-ABI: its potentials equal cfmm_eval's host path
bitwise (same plan, same density; the kernels are deterministic) on two calls
in a row, the second with a smaller plan, and it rejects plans beyond its
static staging."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2509_05458_amd as cf  # noqa: E402


def _abi_static(plan, sig):
    out = np.empty(plan.n_out, dtype=np.complex128)
    s = np.ascontiguousarray(sig, dtype=np.complex128)
    rc = cf.lib().cfmm_eval_static(plan._handle, s.ctypes.data, out.ctypes.data)
    assert rc == cf.CFMM_OK, cf.lib().cfmm_last_error().decode()
    return out


def _abi_host(plan, sig):
    out = np.empty(plan.n_out, dtype=np.complex128)
    s = np.ascontiguousarray(sig, dtype=np.complex128)
    rc = cf.lib().cfmm_eval(plan._handle, s.ctypes.data, out.ctypes.data, 0)
    assert rc == cf.CFMM_OK, cf.lib().cfmm_last_error().decode()
    return out


@pytest.mark.parametrize("ci,kern,n1,n2", [(2, "laplace", 48 * 48, 24 * 24), (0, "helmholtz", 4096, 700),
                                           (3, "helmholtz", 40 * 40, 20 * 20)])
def test_static_eval_equals_host_eval_twice(ci, kern, n1, n2):
    print(f"[gpu] no-alloc {kern} config {ci}: n={n1} then n={n2}", flush=True)
    for n in (n1, n2):                         # the second call is smaller
        cfg = synth.make_config(ci, n=n)
        plan = cf.Plan(cfg.points, kern, cfg.kappa, 1e-6)
        a = _abi_static(plan, cfg.sigma)
        b = _abi_host(plan, cfg.sigma)
        assert np.array_equal(a, b)
        plan.close()


def test_static_eval_with_targets():
    cfg = synth.make_config(0, n=3000)
    trg = synth.curve2d(1234, 9300)
    plan = cf.Plan(cfg.points, "helmholtz", 10.0, 1e-8, targets=trg)
    a = _abi_static(plan, cfg.sigma)
    b = _abi_host(plan, cfg.sigma)
    assert a.shape == (1234,) and np.array_equal(a, b)


def test_static_eval_rejects_plans_beyond_its_staging():
    # 2,099,601 sources, targets = sources: n_src + n_out > 2^22
    m = 1449
    pts = synth.plane3d_grid(m)
    print(f"[gpu] no-alloc size limit n={pts.shape[0]}", flush=True)
    plan = cf.Plan(torch.from_numpy(pts).cuda(), "laplace", 0.0, 1e-3)
    sig = np.zeros(pts.shape[0], np.complex128)
    out = np.empty(pts.shape[0], np.complex128)
    rc = cf.lib().cfmm_eval_static(plan._handle, sig.ctypes.data, out.ctypes.data)
    assert rc == cf.CFMM_EINVAL
    assert "static staging" in cf.lib().cfmm_last_error().decode()
