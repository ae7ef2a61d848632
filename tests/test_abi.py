"""CPU checks of the library: it loads, exports every declared symbol, rejects
invalid arguments before touching a GPU, and its host planning logic (tree,
Lists 1-4, expansion lengths) equals the oracle's bit for bit."""
import os
import re

import numpy as np
import pytest

import paper_2509_05458_amd as cf
import synth
from oracle import params
from oracle import tree as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cfmm.h")).read()
    return sorted(set(re.findall(r"\b(cfmm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = cf.lib()
    names = _declared()
    assert "cfmm_plan" in names and "cfmm_eval" in names and "cfmm_destroy" in names
    for name in names:
        assert hasattr(L, name), name


_PTS = np.zeros((4, 3), np.complex128)


@pytest.mark.parametrize("bad", [
    dict(dim=4), dict(kernel=7), dict(tol=0.0), dict(tol=2.0), dict(n_src=0), dict(wavenumber=-1.0),
    dict(precision=5), dict(separation=3), dict(leaf_size=-2), dict(m2l_form=2), dict(m2l_form=-1),
    # below each kernel's accuracy floor
    dict(tol=1e-13), dict(dim=3, kernel=cf.LAPLACE, tol=1e-13), dict(dim=3, tol=1e-11),
    # mixed precision below its FP32 rounding floor
    dict(precision=cf.MIXED, tol=1e-8), dict(dim=3, kernel=cf.LAPLACE, precision=cf.MIXED, tol=1e-7),
    # targets: a count without points is fine (ignored), points without a count is not
    dict(n_trg=0, trg=_PTS.ctypes.data), dict(n_trg=-3, trg=_PTS.ctypes.data),
    dict(n_src=2 ** 30, n_trg=2 ** 30, trg=_PTS.ctypes.data), dict(src=None)])
def test_invalid_arguments_rejected(bad):
    import ctypes
    kw = dict(dim=2, kernel=cf.HELMHOLTZ, wavenumber=1.0, tol=1e-6, n_src=4, src=_PTS.ctypes.data,
              n_trg=0, trg=None, points_on_device=0, precision=0, stream=None, leaf_size=0, separation=0)
    kw.update(bad)
    d = cf.PlanDesc(**kw)
    h = ctypes.c_void_p()
    rc = cf.lib().cfmm_plan(ctypes.byref(h), ctypes.byref(d))
    assert rc == cf.CFMM_EINVAL
    assert cf.lib().cfmm_last_error().decode() != ""
    assert not h.value


def test_accuracy_floors_match_the_binding():
    src = open(os.path.join(ROOT, "include", "cfmm.h")).read()
    vals = dict(re.findall(r"#define (CFMM_(?:TOL_MIN_\w+|MIXED_TOL_MIN)) ([0-9.e-]+)", src))
    assert float(vals["CFMM_TOL_MIN_HELMHOLTZ_2D"]) == cf.TOL_MIN[(2, "helmholtz")]
    assert float(vals["CFMM_TOL_MIN_LAPLACE_2D"]) == cf.TOL_MIN[(2, "laplace")]
    assert float(vals["CFMM_TOL_MIN_LAPLACE_3D"]) == cf.TOL_MIN[(3, "laplace")]
    assert float(vals["CFMM_TOL_MIN_HELMHOLTZ_3D"]) == cf.TOL_MIN[(3, "helmholtz")]
    assert float(vals["CFMM_MIXED_TOL_MIN"]) == cf.MIXED_TOL_MIN


def test_binding_rejects_bad_points_before_the_library():
    with pytest.raises(ValueError):
        cf.Plan(np.zeros(5, np.complex128), "helmholtz", 1.0, 1e-6)
    with pytest.raises(ValueError):
        cf.Plan(np.zeros((5, 2), np.complex128), "helmholtz", 1.0, 1e-6,
                targets=np.zeros((5, 3), np.complex128))


def test_null_arguments_rejected():
    import ctypes
    L = cf.lib()
    assert L.cfmm_plan(None, None) == cf.CFMM_EINVAL
    h = ctypes.c_void_p()
    assert L.cfmm_plan(ctypes.byref(h), None) == cf.CFMM_EINVAL
    assert L.cfmm_eval(None, None, None, 0) == cf.CFMM_EINVAL
    assert L.cfmm_plan_m2l_work(None, None) == cf.CFMM_EINVAL
    assert L.cfmm_destroy(None) == cf.CFMM_OK


def _cases():
    from tests.test_tree_oracle import CASES
    return CASES


@pytest.mark.parametrize("top", [0, 2, 3])
@pytest.mark.parametrize("case", range(6))
def test_host_tree_and_lists_equal_oracle(case, top):
    name, make, ns, k = _cases()[case]
    pts = make()
    t = T.build_tree(pts, ns, k, top)
    h = cf.host_tree(pts.shape[1], t.keys, ns, k, top)
    for key in ("level", "parent", "child0", "nchild", "pbeg", "pend", "prefix"):
        assert np.array_equal(getattr(t, key).astype(h[key].dtype), h[key]), key
    for q in range(1, 5):
        o, i = t.lists[f"L{q}"]
        ho, hi = h[f"L{q}"]
        assert np.array_equal(o, ho) and np.array_equal(i, hi), q


def test_host_tree_full_size_curve_equals_oracle():
    c = synth.make_config(1, n=1 << 17)
    t = T.build_tree(c.points, 64, 1, 3)
    h = cf.host_tree(2, t.keys, 64, 1, 3)
    assert np.array_equal(t.pbeg, h["pbeg"]) and np.array_equal(t.level, h["level"])
    for q in range(1, 5):
        assert np.array_equal(t.lists[f"L{q}"][1], h[f"L{q}"][1])


@pytest.mark.parametrize("eps", [1e-5, 1e-7, 1e-11, 1e-13])
@pytest.mark.parametrize("w", [1e-3, 0.05, 0.4, 2.0, 5.0])
@pytest.mark.parametrize("sep", [1, 2])
def test_nterms_equals_oracle_rule(eps, w, sep):
    kappa = 10.0
    got = cf.nterms(2, "helmholtz", kappa, w, sep, eps, 63)
    ref = params.nterms(2, "helmholtz", kappa, w, sep, eps, 63)
    assert got == ref


@pytest.mark.parametrize("eps", [1e-6, 1e-10, 1e-12])
@pytest.mark.parametrize("w", [0.01, 0.1875, 0.75, 1.5])
@pytest.mark.parametrize("sep", [1, 2])
def test_nterms_3d_helmholtz_equals_oracle_rule(eps, w, sep):
    kappa = 20.0 * 2.0 * np.pi / 12.0
    got = cf.nterms(3, "helmholtz", kappa, w, sep, eps, 50)
    ref = params.nterms(3, "helmholtz", kappa, w, sep, eps, 50)
    assert got == ref


@pytest.mark.parametrize("kappa", [1e-6, 1e-3, 0.3])
@pytest.mark.parametrize("sep", [1, 2])
def test_nterms_3d_helmholtz_low_frequency_equals_oracle_rule(kappa, sep):
    # small kappa w: |h_n| and j_n leave the FP64 range well before n = 50
    for eps in (1e-6, 1e-10):
        got = cf.nterms(3, "helmholtz", kappa, 1.0, sep, eps, 50)
        ref = params.nterms(3, "helmholtz", kappa, 1.0, sep, eps, 50)
        assert got == ref, (eps, got, ref)


def test_2d_laplace_floor_rejected():
    import ctypes
    pts = np.zeros((4, 2), np.complex128)
    d = cf.PlanDesc(dim=2, kernel=cf.LAPLACE, wavenumber=0.0, tol=1e-13, n_src=4, src=pts.ctypes.data,
                    n_trg=0, trg=None, points_on_device=0, precision=0, stream=None, leaf_size=0,
                    separation=0)
    h = ctypes.c_void_p()
    assert cf.lib().cfmm_plan(ctypes.byref(h), ctypes.byref(d)) == cf.CFMM_EINVAL
    assert not h.value
