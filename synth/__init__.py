"""Seeded synthetic inputs for the complex-coordinate FMM.

This module only draws numbers: it holds none of the method's arithmetic
(no kernel, no expansion, no tree).  Both the oracle tests and the HIP path
consume exactly these arrays.

Geometry families (stand-ins for the paper's timing geometries, Sec. 7.1,
whose panel discretisations are not reproducible here):

* 2D complexified curve  x(t) = (t + i psi(t), 0.2 exp(-t^2)),  t ~ U[-8, 8]
* 3D complexified plane  x(s,t) = (s + i psi(s), t + i psi(t), h(s,t))

with psi(t) = 0.5 * softplus(|t| - 4): zero in the middle, slope <= 0.5, so
the imaginary parts are a Lipschitz function of the real parts with L <= 0.5
(the geometric assumption of Sec. 4.1 / 5.1).

Densities are standard complex Gaussians, Re and Im i.i.d. N(0, 1).
All draws use numpy's PCG64 (``numpy.random.default_rng``), so the arrays are
identical on every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# seeds: geometry 1000+i, density 2000+i, sampled oracle targets 3000+i
GEOM_SEED = 1000
SIGMA_SEED = 2000
TARGET_SEED = 3000


def psi(t):
    """Complexification profile 0.5*softplus(|t|-4) (Lipschitz constant 0.5)."""
    t = np.asarray(t, dtype=np.float64)
    return 0.5 * np.logaddexp(0.0, np.abs(t) - 4.0)


def curve2d(n: int, seed: int, scale: float = 1.0, amp: float = 1.0) -> np.ndarray:
    """n points on the complexified 2D curve, complex128[n, 2]; amp scales the
    imaginary part (Lipschitz constant 0.5 amp)."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(-8.0, 8.0, size=n)
    x = np.empty((n, 2), dtype=np.complex128)
    x[:, 0] = t + 1j * amp * psi(t)
    x[:, 1] = 0.2 * np.exp(-t * t)
    return x * scale


def curve2d_literal(n: int, seed: int, kappa: float, ppw: float = 10.0) -> np.ndarray:
    """The curve family with t ~ U[-L, L] sized for ppw points per wavelength
    (2L = n lambda / ppw): the literal large-N recipe, whose imaginary parts
    reach 0.5 (L - 4), far beyond what e^{kappa Im r} allows in FP64."""
    lam = 2.0 * math.pi / kappa
    L = n * lam / (2.0 * ppw)
    rng = np.random.default_rng(seed)
    t = rng.uniform(-L, L, size=n)
    x = np.empty((n, 2), dtype=np.complex128)
    x[:, 0] = t + 1j * psi(t)
    x[:, 1] = 0.2 * np.exp(-t * t)
    return x


def plane3d_grid(m: int, lo: float = -6.0, hi: float = 6.0) -> np.ndarray:
    """m*m grid points on the complexified plane with height 0.3 exp(-(s^2+t^2))."""
    g = lo + (hi - lo) * np.arange(m, dtype=np.float64) / (m - 1)
    s, t = np.meshgrid(g, g, indexing="ij")
    s = s.ravel()
    t = t.ravel()
    x = np.empty((s.size, 3), dtype=np.complex128)
    x[:, 0] = s + 1j * psi(s)
    x[:, 1] = t + 1j * psi(t)
    x[:, 2] = 0.3 * np.exp(-(s * s + t * t))
    return x


def plane3d_bumps(m: int, seed: int, lo: float = -6.0, hi: float = 6.0,
                  nbumps: int = 8, scale: float = 1.0, amp: float = 1.0) -> np.ndarray:
    """m*m grid on the complexified plane, height = sum of nbumps seeded Gaussians;
    amp scales the imaginary parts."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-4.0, 4.0, size=(nbumps, 2))
    w = rng.uniform(0.5, 2.0, size=nbumps)
    g = lo + (hi - lo) * np.arange(m, dtype=np.float64) / (m - 1)
    s, t = np.meshgrid(g, g, indexing="ij")
    s = s.ravel()
    t = t.ravel()
    h = np.zeros_like(s)
    for b in range(nbumps):
        h += 0.3 * np.exp(-((s - c[b, 0]) ** 2 + (t - c[b, 1]) ** 2) / (w[b] ** 2))
    x = np.empty((s.size, 3), dtype=np.complex128)
    x[:, 0] = s + 1j * amp * psi(s)
    x[:, 1] = t + 1j * amp * psi(t)
    x[:, 2] = h
    return x * scale


def density(n: int, seed: int) -> np.ndarray:
    """Standard complex Gaussian densities, complex128[n]."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


def sample_targets(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct, sorted indices in [0, n) (the sampled oracle targets)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


@dataclass
class Config:
    name: str
    dim: int
    kernel: str            # "helmholtz" or "laplace"
    kappa: float
    tol: float
    points: np.ndarray     # complex128[n, dim]; targets = sources
    sigma: np.ndarray      # complex128[n]
    oracle_targets: np.ndarray  # indices into points for the sampled oracle
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.points.shape[0]


# Config recipes. n may be shrunk (same family, same seeds) for fast tests.
KAPPA_C3 = 20.0 * 2.0 * math.pi / 12.0


def make_config(i: int, n: int | None = None, n_oracle: int = 4096) -> Config:
    if i == 0:
        n = 4096 if n is None else n
        pts = curve2d(n, GEOM_SEED + 0)
        sig = density(n, SIGMA_SEED + 0)
        tg = np.arange(n, dtype=np.int64) if n <= 4096 else sample_targets(n, n_oracle, TARGET_SEED + 0)
        return Config("c0_h2d_4096", 2, "helmholtz", 10.0, 1e-10, pts, sig, tg,
                      {"curve": "t~U[-8,8]", "scale": 1.0})
    if i == 1:
        n = (1 << 20) if n is None else n
        pts = curve2d(n, GEOM_SEED + 1, scale=0.1)
        sig = density(n, SIGMA_SEED + 1)
        tg = sample_targets(n, n_oracle, TARGET_SEED + 1)
        return Config("c1_h2d_1m", 2, "helmholtz", 100.0, 1e-6, pts, sig, tg,
                      {"curve": "t~U[-8,8]", "scale": 0.1})
    if i == 2:
        m = 1448 if n is None else int(round(math.sqrt(n)))
        pts = plane3d_grid(m)
        nn = pts.shape[0]
        sig = density(nn, SIGMA_SEED + 2)
        tg = sample_targets(nn, n_oracle, TARGET_SEED + 2)
        return Config("c2_l3d_2m", 3, "laplace", 0.0, 1e-6, pts, sig, tg,
                      {"grid": m})
    if i == 3:
        m = 1000 if n is None else int(round(math.sqrt(n)))
        pts = plane3d_bumps(m, GEOM_SEED + 3)
        nn = pts.shape[0]
        sig = density(nn, SIGMA_SEED + 3)
        tg = sample_targets(nn, n_oracle, TARGET_SEED + 3)
        return Config("c3_h3d_1m", 3, "helmholtz", KAPPA_C3, 1e-10, pts, sig, tg,
                      {"grid": m})
    raise ValueError(f"no config {i}")


@dataclass
class Request:
    """One served request: a geometry, a wavenumber and a tolerance, evaluated
    for `nmat` densities in turn (the matvecs of an iterative solve).  Arrays
    are drawn on demand from the request's seeds."""
    rid: int
    arrival: float        # seconds after trace start
    dim: int
    kappa: float
    tol: float
    n: int                # number of points (3D: a square grid, n = m^2)
    scale: float          # geometry scale (keeps kappa * extent in the validated range)
    nmat: int = 20

    def points(self) -> np.ndarray:
        if self.dim == 2:
            return curve2d(self.n, 5000 + self.rid, scale=self.scale)
        m = int(round(math.sqrt(self.n)))
        return plane3d_bumps(m, 5000 + self.rid, scale=self.scale)

    def density_factors(self):
        """(a, b): the m-th density is a * exp(2 pi i m b), a complex Gaussian
        (seed 6000 + rid), b uniform on [0, 1) (seed 8000 + rid)."""
        a = density(self.n, 6000 + self.rid)
        b = np.random.default_rng(8000 + self.rid).uniform(0.0, 1.0, size=self.n)
        return a, b

    def density(self, m: int) -> np.ndarray:
        a, b = self.density_factors()
        return a * np.exp(2j * np.pi * m * b)

    def check_targets(self, k: int = 64) -> np.ndarray:
        return sample_targets(self.n, min(k, self.n), 7000 + self.rid)


def serving_trace(nreq: int = 512, rate: float = 100.0, nmat: int = 20,
                  nmin_log2: float = 10.0, nmax_log2: float = 18.0, seed: int = 4000) -> list:
    """Seeded request trace for the served stream: Poisson arrivals at `rate`/s,
    sizes log-uniform in [2^nmin_log2, 2^nmax_log2], half 2D and half 3D
    Helmholtz, kappa log-uniform in [1, 200], tolerance from {1e-4, 1e-6, 1e-10}.
    2D requests use the curve scaled by min(1, 10/kappa); 3D requests the bump
    plane (n = round(sqrt N)^2) scaled by min(1, KAPPA_C3/kappa), so every
    request keeps the wavelength count of the validated configurations."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=nreq)
    arr = np.cumsum(gaps) - gaps[0]
    logn = rng.uniform(nmin_log2, nmax_log2, size=nreq)
    dims = np.where(rng.uniform(size=nreq) < 0.5, 2, 3)
    kap = np.exp(rng.uniform(0.0, math.log(200.0), size=nreq))
    tols = np.array([1e-4, 1e-6, 1e-10])[rng.integers(0, 3, size=nreq)]
    out = []
    for r in range(nreq):
        n = int(round(2.0 ** logn[r]))
        if dims[r] == 2:
            sc = min(1.0, 10.0 / kap[r])
        else:
            m = max(2, int(round(math.sqrt(n))))
            n = m * m
            sc = min(1.0, KAPPA_C3 / kap[r])
        out.append(Request(r, float(arr[r]), int(dims[r]), float(kap[r]), float(tols[r]), n, sc, nmat))
    return out
