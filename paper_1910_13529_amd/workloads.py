"""Grids and solver coefficients of the synthetic workloads (host set-up).

The batched workload draws per-run sizes, gamma and dt/dx1 from
inputs.batch_draws and applies the stability rule used for it: dx1 = 0.05,
dt = (dt/dx1) dx1, sigma1 = max_k (dt/2)[k]_1 (dt/dx1 for Yee; from the
run's own App. C fit at kappa = dx1/dt for the customized solver, M = 16),
customized draws with sigma1 >= 0.995 rejected in favour of the next
candidate, and dx2 = max(dx1, dt / sqrt((1 - sigma1^2) / 2)), which keeps
the 2D Courant number at sqrt((1 + sigma1^2) / 2) < 1.
"""
import math

import numpy as np

from . import inputs

DX1 = 0.05
SIGMA1_MAX = 0.995


def axial_sigma(C, ratio, nq=4000):
    """max over k of (dt/2)[k]_1 for coefficients C at dt/dx1 = ratio"""
    th = np.linspace(0.0, math.pi / 2, nq + 1)
    l = np.arange(1, len(C) + 1)
    v = np.sin(np.outer(th, 2 * l - 1)) @ np.asarray(C, dtype=np.float64)
    return ratio * float(v.max())


def batch_workload(nruns=256, seed=4, solver="mixed", npart=4096, M=16, fit=None, n1_range=(128, 1024),
                   n2_range=(64, 256)):
    """List of run dicts: grid (for relpic), C (None = Yee), particles
    (cell, offset, u), Q per macro-particle, and the draws.  `fit(kappa, M)`
    returns App. C coefficients (default: the library's fit)."""
    if fit is None:
        from .relpic import relpic_fit_coefficients

        def fit(kappa, M):
            return relpic_fit_coefficients(kappa, M)[0]
    runs = []
    for d in inputs.batch_draws(nruns, seed, solver, n1_range=n1_range, n2_range=n2_range):
        chosen = None
        for ratio in d["ratios"]:
            C = None
            sigma1 = ratio
            if d["kind"] == "custom":
                C = np.asarray(fit(1.0 / ratio, M), dtype=np.float64)
                sigma1 = axial_sigma(C, ratio)
                if sigma1 >= SIGMA1_MAX:
                    continue
            chosen = (ratio, C, sigma1)
            break
        if chosen is None:
            raise RuntimeError("no stable dt/dx1 among the candidates of run seed %d" % d["seed"])
        ratio, C, sigma1 = chosen
        dt = ratio * DX1
        dx2 = max(DX1, dt / math.sqrt(0.5 * (1.0 - sigma1 * sigma1)))
        cell, off, u = inputs.batch_bunch(d, npart)
        # peak line density n_b = 1: Q = -(2 pi) sigma1 sigma2 / N (sigma in physical units)
        Q = -2.0 * math.pi * (5.0 * DX1) * (1.0 * dx2) / npart
        grid = dict(ndim=2, n=(d["n1"], d["n2"], 1), dx=(DX1, dx2, 1.0), dt=dt, window=False)
        runs.append({"grid": grid, "C": C, "cell": cell, "offset": off, "u": u, "Q": Q, "sigma1": sigma1,
                     "draw": d})
    return runs


def adjoint_workload(n=(1024, 256), npart=1 << 16, nsteps=200, M=4, fit=None):
    """The differentiable case: 2D periodic grid, dx = 0.05, dt = dx/4
    (kappa = 4), a ballistic bunch of npart particles with gamma = 1e4
    (sigma_z = 0.1, sigma_r = 0.05, centred on the middle node), M axial
    coefficients initialized by the App. C fit (p = 2, w = 0.6, n = 10), the
    loss box 3 sigma around the bunch moving at beta."""
    if fit is None:
        from .relpic import relpic_fit_coefficients

        def fit(kappa, M):
            return relpic_fit_coefficients(kappa, M)[0]
    dx = 0.05
    dt = dx / 4.0
    gamma = 1e4
    sz, sr = 0.1, 0.05
    center = (n[0] // 2, n[1] // 2)
    cell, off, u = inputs.gaussian_bunch(11, npart, center, (sz / dx, sr / dx), gamma, ndim=2, clip_sigmas=4.0)
    beta = math.sqrt(1.0 - 1.0 / (gamma * gamma))
    Q = -2.0 * math.pi * sz * sr / npart  # peak line density 1
    box = dict(x1=center[0] * dx, x2=center[1] * dx, v1=beta, half1=3 * sz, half2=3 * sr)
    grid = dict(ndim=2, n=(n[0], n[1], 1), dx=(dx, dx, 1.0), dt=dt, window=False)
    C0 = np.asarray(fit(dx / dt, M), dtype=np.float64) if M > 1 else np.ones(1)
    return {"grid": grid, "C0": C0, "cell": cell, "offset": off, "u": u, "Q": Q, "box": box, "nsteps": nsteps}
