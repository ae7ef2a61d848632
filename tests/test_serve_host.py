"""CPU checks of the serving layer: trace recipe, precision policy,
admission estimate."""
import math

import numpy as np

import synth
from paper_2509_05458_amd import serve


def test_trace_recipe():
    tr = synth.serving_trace(512)
    assert len(tr) == 512
    arr = np.array([r.arrival for r in tr])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    dims = np.array([r.dim for r in tr])
    assert abs((dims == 2).mean() - 0.5) < 0.08
    ns = np.array([r.n for r in tr])
    assert ns.min() >= 2 ** 10 * 0.9 and ns.max() <= 2 ** 18 * 1.01
    for r in tr:
        if r.dim == 3:
            m = int(round(math.sqrt(r.n)))
            assert m * m == r.n
        assert 1.0 <= r.kappa <= 200.0
        assert r.tol in (1e-4, 1e-6, 1e-10)
        lim = 10.0 if r.dim == 2 else synth.KAPPA_C3
        assert math.isclose(r.scale, min(1.0, lim / r.kappa))


def test_request_arrays_are_seeded_and_new_per_matvec():
    r = synth.serving_trace(4)[1]
    p1, p2 = r.points(), r.points()
    assert np.array_equal(p1, p2) and p1.shape == (r.n, r.dim)
    d0, d1 = r.density(0), r.density(1)
    assert np.array_equal(d0, r.density(0)) and not np.allclose(d0, d1)
    a, b = r.density_factors()
    assert np.allclose(d1, a * np.exp(2j * np.pi * b))


def test_precision_policy():
    assert serve.precision_for(1e-4) == "mixed"
    assert serve.precision_for(1e-6) == "mixed"
    assert serve.precision_for(1e-10) == "fp64"


def test_estimate_grows_with_n():
    assert serve.estimate_bytes(2, 1 << 18) > serve.estimate_bytes(2, 1 << 10)
    assert serve.estimate_bytes(3, 1 << 16) > serve.estimate_bytes(2, 1 << 16)
