"""Pins of the oracle's 3D layer potentials (Sec. 2.1: double layer with
dipole vectors v = tau nu, and the gradients behind the normal derivatives)
against what fixes them independently of its formulas: central differences of
the single-layer oracle in the source and target positions (G is analytic in
every coordinate, so a complex step direction is allowed), the textbook
real-coordinate kernels, and the identity grad_x G = -grad_y G between its
two code paths."""
import numpy as np
import pytest

import oracle
import synth


def _pts(n, seed, c=0.0):
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1, 1, (n, 3)) + c
    return re + 0.2j * np.sin(re[:, [1, 2, 0]])


@pytest.mark.parametrize("kernel,kappa", [("laplace", 0.0), ("helmholtz", 3.0)])
def test_dipole_is_the_directional_derivative_in_the_source(kernel, kappa):
    x = _pts(20, 1, 3.0)
    y = _pts(1, 2)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    h = 1e-5
    u, _ = oracle.layer3(kernel, kappa, x, y, dipole=v[None, :])
    one = np.ones(1, np.complex128)
    fd = (oracle.direct(3, kernel, kappa, x, y + h * v, one) - oracle.direct(3, kernel, kappa, x, y - h * v, one)) / (2 * h)
    assert np.allclose(u, fd, rtol=1e-8, atol=0)


@pytest.mark.parametrize("kernel,kappa", [("laplace", 0.0), ("helmholtz", 3.0)])
def test_gradient_is_the_derivative_in_the_target(kernel, kappa):
    x = _pts(15, 4, 3.0)
    y = _pts(30, 5)
    rng = np.random.default_rng(6)
    q = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    v = rng.standard_normal((30, 3)) + 1j * rng.standard_normal((30, 3))
    h = 1e-5
    _, g = oracle.layer3(kernel, kappa, x, y, charge=q, dipole=v)
    for k in range(3):
        for step in (h, 1j * h):      # real and imaginary directions (holomorphy)
            e = np.zeros(3, np.complex128)
            e[k] = step
            up, _ = oracle.layer3(kernel, kappa, x + e, y, charge=q, dipole=v)
            um, _ = oracle.layer3(kernel, kappa, x - e, y, charge=q, dipole=v)
            fd = (up - um) / (2 * step)
            assert np.allclose(g[:, k], fd, rtol=1e-7, atol=0), (k, step)


def test_real_coordinates_give_the_textbook_laplace_kernels():
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, (10, 3)) + 3.0
    y = rng.uniform(-1, 1, (12, 3))
    v = rng.standard_normal((12, 3))
    u, g = oracle.layer3("laplace", 0.0, x + 0j, y + 0j, dipole=v + 0j)
    d = x[:, None, :] - y[None, :, :]
    r = np.linalg.norm(d, axis=2)
    vd = np.einsum("ijk,jk->ij", d, v)
    assert np.allclose(u, np.sum(vd / (4 * np.pi * r ** 3), axis=1), rtol=1e-14, atol=0)
    gt = np.sum(v[None, :, :] / (4 * np.pi * r[..., None] ** 3) - 3 * vd[..., None] * d / (4 * np.pi * r[..., None] ** 5), axis=1)
    assert np.allclose(g, gt, rtol=1e-13, atol=1e-15)
    q = rng.standard_normal(12)
    _, g = oracle.layer3("laplace", 0.0, x + 0j, y + 0j, charge=q + 0j)
    gt = np.sum(-q[None, :, None] * d / (4 * np.pi * r[..., None] ** 3), axis=1)
    assert np.allclose(g, gt, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kernel,kappa", [("laplace", 0.0), ("helmholtz", 2.0)])
def test_charge_gradient_equals_minus_unit_dipole(kernel, kappa):
    # d/dx_k G(x, y) = -d/dy_k G(x, y): the gradient path on a charge and the
    # dipole path on a unit vector must agree
    x = _pts(25, 8, 2.5)
    y = _pts(40, 9)
    q = synth.density(40, 10)
    _, g = oracle.layer3(kernel, kappa, x, y, charge=q)
    for k in range(3):
        v = np.zeros((40, 3), np.complex128)
        v[:, k] = q
        u, _ = oracle.layer3(kernel, kappa, x, y, dipole=v)
        assert np.allclose(g[:, k], -u, rtol=1e-13, atol=1e-16)


def test_charge_potential_equals_direct_sum_and_self_term():
    pts = synth.plane3d_grid(9)
    q = synth.density(pts.shape[0], 11)
    u, _ = oracle.layer3_self("laplace", 0.0, pts, charge=q)
    u0 = oracle.direct_self(3, "laplace", 0.0, pts, q)
    assert np.allclose(u, u0, rtol=1e-14, atol=0)
