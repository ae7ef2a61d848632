"""CPU checks of the GMRES driver (torch on the host, a dense matrix as the
operator, numpy's dense solve as the reference) and of the curve
quadrature nodes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2509_05458_amd import gmres as G  # noqa: E402


def _system(n, seed, scale=0.4):
    rng = np.random.default_rng(seed)
    A = np.eye(n) + scale * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


@pytest.mark.parametrize("restart", [80, 7])
def test_gmres_matches_dense_solve(restart):
    A, b = _system(80, 3)
    At = torch.from_numpy(A)
    x, info = G.gmres(lambda v: At @ v, torch.from_numpy(b), tol=1e-12, restart=restart, maxiter=2000)
    ref = np.linalg.solve(A, b)
    assert info.converged
    assert np.linalg.norm(x.numpy() - ref) / np.linalg.norm(ref) < 1e-10
    # the reported residuals fall and end below tol
    assert info.residuals[-1] <= 1e-12 * 1.01
    if restart < 80:
        assert info.restarts > 1


def test_gmres_exact_in_n_steps_for_low_rank_perturbation():
    # A = I + u v^H: the Krylov space of any b closes after two steps
    rng = np.random.default_rng(4)
    n = 50
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A = np.eye(n) + 0.1 * np.outer(u, v.conj())
    b = rng.standard_normal(n) + 0j
    At = torch.from_numpy(A)
    x, info = G.gmres(lambda w: At @ w, torch.from_numpy(b), tol=1e-13, restart=20)
    assert info.iterations <= 3
    assert np.allclose(x.numpy(), np.linalg.solve(A, b), rtol=1e-11, atol=1e-12)


def test_zero_rhs():
    x, info = G.gmres(lambda v: v, torch.zeros(5, dtype=torch.complex128))
    assert info.converged and info.iterations == 0 and torch.all(x == 0)


def test_curve_nodes_weights_integrate_the_complex_line_element():
    # sum of weights = integral of sqrt(x1'^2 + x2'^2) dt, which for psi = 0
    # and h = 0 is the length 2T; for the complexified curve, by Cauchy, the
    # integral of dx1 along the curve is x1(T) - x1(-T)
    x, w = G.curve_nodes(4001, T=8.0, psi=(lambda t: 0 * t, lambda t: 0 * t),
                         height=(lambda t: 0 * t, lambda t: 0 * t))
    assert abs(w.sum() - 16.0) < 1e-11
    x, w = G.curve_nodes(4001, T=8.0, height=(lambda t: 0 * t, lambda t: 0 * t))
    # with h = 0: sqrt(x1'^2) = x1' (principal, Re > 0), so sum w = x1(T) - x1(-T) to O(dt^2)
    assert abs(w.sum() - (x[-1, 0] - x[0, 0])) < 1e-5
