"""GMRES on the library: iterative solves whose matvecs are cfmm evaluations.

The iterative solves the complex-coordinate FMM serves (Sec. 2.2: boundary
integral equations on complex-scaled interfaces, solved by GMRES, Sec. 7.2)
apply one plan many times with new densities.  This module is that driver:

* ``gmres(matvec, b, ...)``: restarted GMRES (Saad and Schultz) with
  modified Gram-Schmidt Arnoldi and Givens rotations; the Krylov basis lives
  on the device, the small Hessenberg least-squares problem on the host.
* ``LayerOperator``: the discretised operator a sigma + S[w sigma] of a
  second-kind integral equation, S the single-layer sum of a plan (self term
  left out: the punctured rule) and w the quadrature weights of the nodes,
  so that one application is one cfmm_eval.
* ``curve_nodes``: nodes and complex arc-length weights of a complexified
  curve x(t) = (t + i psi(t), h(t)) by the trapezoidal rule on [-T, T].

Every arithmetic step of a matvec runs in the HIP library; the GMRES
bookkeeping is torch on the same device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import Plan


@dataclass
class GmresInfo:
    converged: bool
    iterations: int           # matvecs applied
    residuals: list           # relative residual norm after each iteration
    restarts: int


def gmres(matvec, b, x0=None, tol: float = 1e-8, restart: int = 40, maxiter: int = 400):
    """Solve A x = b for complex128 device vectors (torch) with restarted GMRES.

    matvec(v) returns A v (a new tensor).  Stops when ||b - A x|| / ||b|| <= tol
    (the Arnoldi estimate, checked against a true residual at each restart) or
    after maxiter matvecs.  Returns (x, GmresInfo)."""
    import torch
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    bnorm = float(torch.linalg.vector_norm(b))
    if bnorm == 0.0:
        return torch.zeros_like(b), GmresInfo(True, 0, [0.0], 0)
    res_hist = []
    its = 0
    restarts = 0
    while True:
        r = b - matvec(x) if its > 0 or x0 is not None else b.clone()
        beta = float(torch.linalg.vector_norm(r))
        rel = beta / bnorm
        if not res_hist:
            res_hist.append(rel)
        if rel <= tol or its >= maxiter:
            return x, GmresInfo(rel <= tol, its, res_hist, restarts)
        m = min(restart, maxiter - its)
        V = torch.empty((m + 1, b.numel()), dtype=b.dtype, device=b.device)
        V[0] = r / beta
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k_done = 0
        for k in range(m):
            w = matvec(V[k])
            its += 1
            for i in range(k + 1):                      # modified Gram-Schmidt
                h = torch.vdot(V[i], w)
                w = w - h * V[i]
                H[i, k] = complex(h)
            hn = float(torch.linalg.vector_norm(w))
            H[k + 1, k] = hn
            if hn > 0.0:
                V[k + 1] = w / hn
            # apply the previous rotations, then make this column's
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -np.conj(sn[i]) * H[i, k] + np.conj(cs[i]) * H[i + 1, k]
                H[i, k] = t
            a, c = H[k, k], H[k + 1, k]
            den = math.hypot(abs(a), abs(c))
            if den == 0.0:
                cs[k], sn[k] = 1.0, 0.0
            else:
                cs[k] = np.conj(a) / den if a != 0 else 0.0
                sn[k] = np.conj(c) / den
                if a == 0:
                    cs[k], sn[k] = 0.0, 1.0
            H[k, k] = cs[k] * a + sn[k] * c
            H[k + 1, k] = 0.0
            g[k + 1] = -np.conj(sn[k]) * g[k]
            g[k] = cs[k] * g[k]
            k_done = k + 1
            rel = abs(g[k + 1]) / bnorm
            res_hist.append(rel)
            if rel <= tol or hn == 0.0 or its >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done]) if k_done else np.zeros(0)
        yt = torch.from_numpy(y).to(b.device)
        x = x + torch.mv(V[:k_done].transpose(0, 1), yt)
        restarts += 1


class LayerOperator:
    """sigma -> a sigma + S[w sigma] (the plan's targets are its sources)."""

    def __init__(self, plan: Plan, weights, shift: complex):
        import torch
        self.plan = plan
        self.w = weights if hasattr(weights, "is_cuda") else torch.from_numpy(np.asarray(weights))
        self.shift = shift
        self.calls = 0

    def __call__(self, sigma):
        self.calls += 1
        u = self.plan((self.w * sigma).contiguous())
        return self.shift * sigma + u


def curve_nodes(n: int, T: float = 8.0, height=None, psi=None, scale: float = 1.0):
    """n trapezoidal nodes on the complexified curve x(t) = (t + i psi(t), h(t)),
    t in [-T, T], with complex arc-length weights dt * sqrt(x1'(t)^2 + x2'(t)^2)
    (principal root, the complexified line element).  Defaults: psi(t) =
    0.5 softplus(|t| - 4), h(t) = 0.2 exp(-t^2).  Returns (points [n, 2],
    weights [n])."""
    t = np.linspace(-T, T, n)
    dt = t[1] - t[0]
    if psi is None:
        def psi(u):
            return 0.5 * np.logaddexp(0.0, np.abs(u) - 4.0)

        def dpsi(u):
            return 0.5 * np.sign(u) / (1.0 + np.exp(-(np.abs(u) - 4.0)))
    else:
        psi, dpsi = psi
    if height is None:
        def height(u):
            return 0.2 * np.exp(-u * u)

        def dheight(u):
            return -0.4 * u * np.exp(-u * u)
    else:
        height, dheight = height
    x = np.empty((n, 2), dtype=np.complex128)
    x[:, 0] = t + 1j * psi(t)
    x[:, 1] = height(t)
    d1 = 1.0 + 1j * dpsi(t)
    d2 = dheight(t).astype(np.complex128)
    wts = np.sqrt(d1 * d1 + d2 * d2) * dt
    wts[0] *= 0.5
    wts[-1] *= 0.5
    return x * scale, wts * scale
