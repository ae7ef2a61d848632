"""Pins of the oracle's direct sum and special function against what the
mathematics fixes: library Bessel routines (scipy's AMOS and real-axis
routines), 30-digit mpmath brute force, closed forms, symmetry and the
invariances of the complexified distance (Sec. 2.1, Sec. 3.1)."""
import math
import os

import numpy as np
import pytest
import scipy.special as sp

import oracle
import synth

mp = pytest.importorskip("mpmath")
HERE = os.path.dirname(os.path.abspath(__file__))


def _sector(n, rmin, rmax, deg, seed):
    rng = np.random.default_rng(seed)
    r = 10 ** rng.uniform(math.log10(rmin), math.log10(rmax), n)
    th = np.deg2rad(rng.uniform(-deg, deg, n))
    return r * np.exp(1j * th)


def test_h0_against_amos_in_sector():
    z = _sector(40000, 1e-6, 600.0, 60.0, 1)
    z = z[np.abs(z.imag) < 600]
    h = oracle.hankel0(z)
    ref = sp.hankel1(0, z)
    ok = np.isfinite(ref) & (np.abs(ref) > 1e-300)
    err = np.abs(h[ok] - ref[ok]) / np.abs(ref[ok])
    assert np.all(err < 2e-14 + 4.4e-16 * np.abs(z[ok]))
    assert np.median(err) < 2e-15


def test_h0_against_mpmath_30_digits():
    # mpmath forms J + iY, which cancels by exp(2 Im z) when Im z > 0: 50 digits
    # and |Im z| <= 30 keep more than 20 correct digits
    mp.mp.dps = 50
    z = _sector(600, 1e-5, 300.0, 60.0, 2)
    z = z[np.abs(z.imag) <= 30.0]
    h = oracle.hankel0(z)
    ref = np.array([complex(mp.hankel1(0, mp.mpc(v.real, v.imag))) for v in z])
    err = np.abs(h - ref) / np.abs(ref)
    # H0 ~ exp(iz): its condition number in z is |z|, so allow |z| ulps on top
    assert np.all(err < 1e-14 + 2.2e-16 * np.abs(z))


def test_h0_real_axis_is_j0_plus_i_y0():
    x = 10 ** np.linspace(-5, 2.7, 3000)
    h = oracle.hankel0(x.astype(np.complex128))
    ref = sp.j0(x) + 1j * sp.y0(x)
    # absolute error relative to the envelope sqrt(2/(pi x)) near zeros of J0, Y0
    env = np.maximum(np.abs(ref), np.sqrt(2.0 / (np.pi * x)))
    assert np.max(np.abs(h - ref) / env) < 1e-14


def test_h0_series_asymptotic_and_continuation_agree_at_switch_radii():
    # the three regimes join continuously: compare across a tiny step at each switch
    for r in (2.5, 25.0):
        for deg in (-50, -20, 0, 20, 50):
            e = np.exp(1j * np.deg2rad(deg))
            z = np.array([r * (1 - 1e-12) * e, r * (1 + 1e-12) * e])
            h = oracle.hankel0(z)
            # remove the first-order change H0' dz = -H1 dz (library H1)
            jump = h[1] - h[0] + sp.hankel1(1, z[0]) * (z[1] - z[0])
            assert abs(jump) / abs(h[0]) < 1e-14


def _mp_green(dim, kernel, kappa, x, y):
    s = mp.mpc(0)
    for d in range(dim):
        dd = mp.mpc(x[d].real, x[d].imag) - mp.mpc(y[d].real, y[d].imag)
        s += dd * dd
    r = mp.sqrt(s)
    if dim == 2:
        if kernel == "helmholtz":
            return 0.25j * mp.hankel1(0, kappa * r)
        return -mp.log(r) / (2 * mp.pi)
    if kernel == "helmholtz":
        return mp.exp(1j * kappa * r) / (4 * mp.pi * r)
    return 1 / (4 * mp.pi * r)


@pytest.mark.parametrize("dim,kernel,kappa", [(2, "helmholtz", 10.0), (2, "laplace", 0.0),
                                              (3, "laplace", 0.0), (3, "helmholtz", 10.472)])
def test_direct_sum_brute_force_mpmath(dim, kernel, kappa):
    mp.mp.dps = 30
    n = 24
    if dim == 2:
        pts = synth.curve2d(n, 11)
    else:
        pts = synth.plane3d_bumps(5, 12)[:n]
        n = pts.shape[0]
    sig = synth.density(n, 13)
    u = oracle.direct_self(dim, kernel, kappa, pts, sig)
    ref = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        acc = mp.mpc(0)
        for j in range(n):
            if j != i:
                acc += _mp_green(dim, kernel, kappa, pts[i], pts[j]) * mp.mpc(sig[j].real, sig[j].imag)
        ref[i] = complex(acc)
    assert oracle.rel_l2(u, ref) < 1e-14
    assert np.max(np.abs(u - ref) / np.abs(ref)) < 1e-12


def test_real_coordinates_reduce_to_textbook_kernels():
    rng = np.random.default_rng(5)
    x = rng.uniform(-3, 3, (200, 2))
    y = rng.uniform(-3, 3, (200, 2))
    s = np.sum((x - y) ** 2, axis=1).astype(np.complex128)
    dist = np.sqrt(s.real)
    g = oracle.green(2, "helmholtz", 7.0, s)
    assert np.allclose(g, 0.25j * sp.hankel1(0, 7.0 * dist), rtol=1e-13, atol=0)
    g = oracle.green(3, "laplace", 0.0, s)
    assert np.allclose(g, 1.0 / (4 * np.pi * dist), rtol=1e-15, atol=0)
    g = oracle.green(3, "helmholtz", 3.0, s)
    assert np.allclose(g, np.exp(3j * dist) / (4 * np.pi * dist), rtol=1e-14, atol=0)
    g = oracle.green(2, "laplace", 0.0, s)
    assert np.allclose(g, -np.log(dist) / (2 * np.pi), rtol=1e-13, atol=1e-15)


def test_collinear_complex_points_closed_form():
    # x2 = y2 = 0: r^2 = (x1-y1)^2, principal root = +-(x1-y1) with Re > 0
    rng = np.random.default_rng(6)
    a = rng.uniform(-5, 5, 300) + 0.4j * rng.uniform(-1, 1, 300)
    b = rng.uniform(-5, 5, 300) + 0.4j * rng.uniform(-1, 1, 300)
    d = a - b
    d = np.where(d.real >= 0, d, -d)
    g = oracle.green(2, "helmholtz", 4.0, d * d)
    assert np.allclose(g, 0.25j * sp.hankel1(0, 4.0 * d), rtol=1e-13, atol=0)


@pytest.mark.parametrize("dim,kernel,kappa", [(2, "helmholtz", 10.0), (3, "laplace", 0.0),
                                              (3, "helmholtz", 5.0), (2, "laplace", 0.0)])
def test_symmetric_matrix_bitwise(dim, kernel, kappa):
    pts = synth.curve2d(300, 21) if dim == 2 else synth.plane3d_grid(17)
    n = pts.shape[0]
    rng = np.random.default_rng(22)
    for _ in range(20):
        k, l = rng.choice(n, 2, replace=False)
        e_k = np.zeros(n, dtype=np.complex128)
        e_k[k] = 1.0
        e_l = np.zeros(n, dtype=np.complex128)
        e_l[l] = 1.0
        a_lk = oracle.direct_self(dim, kernel, kappa, pts, e_k, targets=[l])[0]
        a_kl = oracle.direct_self(dim, kernel, kappa, pts, e_l, targets=[k])[0]
        assert a_lk == a_kl


def test_complex_translation_and_rotation_invariance():
    pts = synth.plane3d_bumps(12, 31)
    n = pts.shape[0]
    sig = synth.density(n, 32)
    u0 = oracle.direct_self(3, "helmholtz", 4.0, pts, sig)
    c = np.array([0.3 + 0.1j, -0.2 + 0.05j, 0.7 - 0.02j])
    u1 = oracle.direct_self(3, "helmholtz", 4.0, pts + c[None, :], sig)
    assert oracle.rel_l2(u1, u0) < 1e-13
    # complex rotation: exp of a complex antisymmetric matrix is in SO(3)(C)
    from scipy.linalg import expm
    A = np.array([[0, 0.3 + 0.1j, -0.2], [-(0.3 + 0.1j), 0, 0.1 - 0.05j], [0.2, -(0.1 - 0.05j), 0]])
    Q = expm(A)
    assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-14)
    u2 = oracle.direct_self(3, "helmholtz", 4.0, pts @ Q.T, sig)
    assert oracle.rel_l2(u2, u0) < 1e-12


def test_holomorphy_in_each_coordinate():
    rng = np.random.default_rng(41)
    for dim, kernel, kappa in ((2, "helmholtz", 6.0), (3, "laplace", 0.0), (3, "helmholtz", 6.0),
                               (2, "laplace", 0.0)):
        for _ in range(20):
            x = rng.uniform(-1, 1, dim) + 0.2j * rng.uniform(-1, 1, dim)
            y = rng.uniform(-1, 1, dim) + 0.2j * rng.uniform(-1, 1, dim)
            h = 1e-6
            for d in range(dim):
                def g(shift):
                    xx = x.copy()
                    xx[d] += shift
                    return oracle.green(dim, kernel, kappa, np.array([np.sum((xx - y) ** 2)]))[0]
                dre = (g(h) - g(-h)) / (2 * h)
                dim_ = (g(1j * h) - g(-1j * h)) / (2 * h)
                assert abs(dim_ - 1j * dre) <= 1e-6 * (abs(dre) + 1e-3)


def test_helmholtz3d_small_kappa_tends_to_laplace():
    pts = synth.plane3d_grid(9)
    sig = synth.density(pts.shape[0], 51)
    ul = oracle.direct_self(3, "laplace", 0.0, pts, sig)
    uh = oracle.direct_self(3, "helmholtz", 1e-9, pts, sig)
    # e^{i k r} = 1 + O(k r): the difference is first order in kappa
    assert oracle.rel_l2(uh, ul) < 1e-7


def test_self_term_and_coincident_points_contribute_nothing():
    pts = synth.curve2d(50, 61)
    pts2 = np.concatenate([pts, pts[:1]])    # a duplicate of point 0
    sig = synth.density(51, 62)
    u = oracle.direct_self(2, "helmholtz", 3.0, pts2, sig, targets=[0])
    u_ref = oracle.direct_self(2, "helmholtz", 3.0, pts, sig[:50], targets=[0])
    assert u[0] == pytest.approx(u_ref[0], rel=1e-14)


def test_laplace2d_collinear_closed_form_and_split_logs():
    """2D Laplace, G = -(1/2 pi) log r.  On the line x2 = y2 = 0, r = +-(x1 - y1)
    with Re r > 0, so G = -(1/2 pi) Log(+-(x1 - y1)).  Off the line, with
    z = x1 + i x2 and w = x1 - i x2 (independent complex numbers), r^2 =
    (z_x - z_y)(w_x - w_y), and for points close to the real plane the
    principal logs split: log r = (Log dz + Log dw)/2."""
    rng = np.random.default_rng(71)
    a = rng.uniform(-5, 5, 300) + 0.4j * rng.uniform(-1, 1, 300)
    b = rng.uniform(-5, 5, 300) + 0.4j * rng.uniform(-1, 1, 300)
    d = a - b
    d = np.where(d.real >= 0, d, -d)
    g = oracle.green(2, "laplace", 0.0, d * d)
    assert np.allclose(g, -np.log(d) / (2 * np.pi), rtol=1e-14, atol=1e-15)
    x = rng.uniform(-1, 1, (300, 2)) + 0.1j * rng.uniform(-1, 1, (300, 2))
    y = rng.uniform(2, 3, (300, 2)) + 0.1j * rng.uniform(-1, 1, (300, 2))
    dz = (x[:, 0] + 1j * x[:, 1]) - (y[:, 0] + 1j * y[:, 1])
    dw = (x[:, 0] - 1j * x[:, 1]) - (y[:, 0] - 1j * y[:, 1])
    s = np.sum((x - y) ** 2, axis=1)
    assert np.allclose(dz * dw, s, rtol=1e-14)
    g = oracle.green(2, "laplace", 0.0, s)
    assert np.allclose(g, -(np.log(dz) + np.log(dw)) / (4 * np.pi), rtol=1e-13, atol=1e-15)
