"""Seeded synthetic inputs for relativistic-beam PIC runs.

This module only draws random numbers and lays them out; it holds none of
the PIC method's arithmetic, so both the GPU path and its CPU checker can
consume the same inputs.  Positions are returned as (cell, offset) in cell
units: cell = nearest lattice node (int32, x1 global), offset in [-1/2, 1/2).
Offsets are rounded to multiples of 2^-40 so that cell + offset is exact in
FP64 for |cell| < 2^12.

Workloads (all synthetic, shaped like the paper's cases):
  single_particle   one macro-electron on a node moving along +x1
  gaussian_bunch    tri-Gaussian beam: sigma_z, sigma_r, gamma with relative
                    spread, rms divergence (u_perp = u1 * theta)
  plasma_lattice    cold background electrons on a regular sub-lattice with
                    Gaussian thermal momenta
  random_fields     smooth random field arrays for operator tests
"""
from dataclasses import dataclass, field
import math

import numpy as np

Q40 = 2.0 ** -40


def split_positions(X):
    """Absolute positions in cell units -> (cell int32, offset float64)."""
    X = np.asarray(X, dtype=np.float64)
    cell = np.floor(X + 0.5)
    off = np.round((X - cell) / Q40) * Q40
    # rounding may push an offset onto +1/2: move it to the next cell
    hi = off >= 0.5
    cell = cell + hi
    off = off - hi * 1.0
    return cell.astype(np.int32), off


def single_particle(node, gamma, ndim=2):
    cell = np.asarray(node, dtype=np.int32).reshape(1, ndim)
    off = np.zeros((1, ndim))
    u = np.zeros((1, 3))
    u[0, 0] = math.sqrt(gamma * gamma - 1.0)
    return cell, off, u


def gaussian_bunch(seed, npart, center, sigma, gamma, espread=0.0, divergence=0.0, ndim=3,
                   clip_sigmas=None):
    """center, sigma in cell units per dimension (len ndim)."""
    rng = np.random.default_rng(seed)
    center = np.asarray(center, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    z = rng.standard_normal((npart, ndim))
    if clip_sigmas is not None:
        z = np.clip(z, -clip_sigmas, clip_sigmas)
    X = center[None, :] + sigma[None, :] * z
    g = gamma * (1.0 + espread * rng.standard_normal(npart)) if espread else np.full(npart, float(gamma))
    th = divergence * rng.standard_normal((npart, 2)) if divergence else np.zeros((npart, 2))
    p = np.sqrt(g * g - 1.0)
    u = np.empty((npart, 3))
    u[:, 0] = p / np.sqrt(1.0 + th[:, 0] ** 2 + th[:, 1] ** 2)
    u[:, 1] = u[:, 0] * th[:, 0]
    u[:, 2] = u[:, 0] * th[:, 1]
    cell, off = split_positions(X)
    return cell, off, u


def plasma_lattice(seed, lo, hi, ppc, uth, ndim=3):
    """ppc[d] particles per cell per dimension at offsets (a+1/2)/ppc - 1/2,
    covering cells lo[d] <= i < hi[d]; u ~ uth * N(0, 1) per component."""
    rng = np.random.default_rng(seed)
    axes = []
    for d in range(ndim):
        sub = (np.arange(ppc[d]) + 0.5) / ppc[d] - 0.5
        cells = np.arange(lo[d], hi[d])
        axes.append((cells[:, None] + sub[None, :]).reshape(-1))
    grids = np.meshgrid(*axes, indexing="ij")
    X = np.stack([g.reshape(-1) for g in grids], axis=1)
    u = uth * rng.standard_normal((X.shape[0], 3))
    cell, off = split_positions(X)
    return cell, off, u


def uniform_particles(seed, npart, n, uth, ndim=3):
    """npart positions uniform over the grid (cell units; cell i covers
    [i - 1/2, i + 1/2), i = 0 .. n[d] - 1), u ~ uth * N(0, 1) per component,
    in the order drawn (not cell-sorted)."""
    rng = np.random.default_rng(seed)
    nn = np.asarray(n[:ndim], dtype=np.float64)[None, :]
    X = np.minimum(rng.uniform(0.0, 1.0, (npart, ndim)) * nn - 0.5, nn - 0.5 - 1e-6)
    u = uth * rng.standard_normal((npart, 3))
    cell, off = split_positions(X)
    return cell, off, u


def cells_with_counts(seed, counts, uth):
    """counts[i1, i2, (i3)] particles in each cell, uniform inside it; u ~
    uth * N(0, 1) per component; returned in a random order (not
    cell-sorted)."""
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts, dtype=np.int64)
    ndim = counts.ndim
    idx = np.repeat(np.arange(counts.size), counts.ravel())
    base = np.stack(np.unravel_index(idx, counts.shape), axis=1).astype(np.float64)
    X = base + rng.uniform(-0.5, 0.5, base.shape)
    X = np.minimum(X, base + 0.5 - 1e-6)
    perm = rng.permutation(len(X))
    cell, off = split_positions(X[perm])
    u = uth * rng.standard_normal((len(X), 3))
    return cell[:, :ndim], off[:, :ndim], u


def random_fields(seed, shape, scale=1.0, ncomp=6):
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal(shape) for _ in range(ncomp)]


@dataclass
class Workload:
    """One PIC configuration (fields in the units of the paper: c = 1, lengths
    in c/omega_p, time in 1/omega_p)."""
    name: str
    ndim: int
    n: tuple
    dx: tuple
    dt: float
    window: bool
    solver: str  # "yee" or "custom"
    steps: int
    extra: dict = field(default_factory=dict)


def config_single_particle():
    """2D 256x128, dx = 0.05, dt = 0.9 x Courant, one electron gamma = 1000 at node (64, 64)."""
    dx = 0.05
    dt = 0.9 * dx / math.sqrt(2.0)
    return Workload("single-particle-2d", 2, (256, 128), (dx, dx), dt, False, "yee", 400,
                    {"gamma": 1000.0, "node": (64, 64)})


def config_beam3d(solver="yee", n=(512, 256, 256), npart=1 << 22):
    """3D vacuum beam in a moving window: dx = (0.02, 0.05, 0.05), kappa = 4."""
    dx = (0.02, 0.05, 0.05)
    dt = dx[0] / 4.0
    return Workload("beam-3d-%s" % solver, 3, tuple(n), dx, dt, True, solver, 1000,
                    {"npart": npart, "center": (0.75 * n[0], n[1] / 2, n[2] / 2),
                     "sigma_phys": (0.1, 0.05, 0.05), "gamma": 1e4, "espread": 0.01, "divergence": 1e-3,
                     "n_peak": 100.0})


def beam_inputs(w, seed=2):
    e = w.extra
    sigma = [e["sigma_phys"][d] / w.dx[d] for d in range(w.ndim)]
    return gaussian_bunch(seed, e["npart"], e["center"], sigma, e["gamma"], e["espread"], e["divergence"],
                          ndim=w.ndim, clip_sigmas=4.0)


def beam_charge(w):
    """Macro-particle charge for a peak density n_peak n0 (electrons: negative)."""
    e = w.extra
    vol = (2.0 * math.pi) ** 1.5 * e["sigma_phys"][0] * e["sigma_phys"][1] * e["sigma_phys"][2]
    return -e["n_peak"] * vol / e["npart"]


def batch_draws(nruns=256, seed=4, solver="mixed", spare=8, n1_range=(128, 1024), n2_range=(64, 256)):
    """Per-run draws of the batched workload: n1 ~ U{128..1024}, n2 ~ U{64..256}
    (other inclusive ranges for smaller test cases),
    gamma log-uniform on [10, 1e5], `spare` candidates of dt/dx1 ~ U[0.3, 0.99]
    (a run takes the first one its stability rule accepts), the solver kind
    ("yee" or "custom"; "mixed" draws it per run) and the seed of its bunch."""
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(nruns):
        n1 = int(rng.integers(n1_range[0], n1_range[1] + 1))
        n2 = int(rng.integers(n2_range[0], n2_range[1] + 1))
        gamma = float(10.0 ** rng.uniform(1.0, 5.0))
        ratios = rng.uniform(0.3, 0.99, size=spare)
        flip = rng.random()
        kind = solver if solver in ("yee", "custom") else ("yee" if flip < 0.5 else "custom")
        runs.append({"n1": n1, "n2": n2, "gamma": gamma, "ratios": ratios, "kind": kind,
                     "seed": seed * 1000003 + r})
    return runs


def batch_bunch(run, npart=4096, sigma_cells=(5.0, 1.0)):
    """Gaussian bunch of one batched run in cell units: centred at 3/4 of n1
    on the middle x2 node, sigma 5 cells along x1 and 1 cell along x2,
    u1 = sqrt(gamma^2 - 1), no transverse momentum."""
    center = (0.75 * run["n1"], run["n2"] // 2)
    return gaussian_bunch(run["seed"], npart, center, sigma_cells, run["gamma"], ndim=2, clip_sigmas=4.0)


def config_drift3d(n=(256, 120, 120)):
    """The paper's drifting-beam sample (Sec. 3.1): a tri-Gaussian electron
    beam of 1 GeV (gamma = 1957), peak density n_b = 100 n_p, k_p sigma_z = 1,
    k_p sigma_r = 0.5, no emittance or energy spread, in free space; dx1 = 0.05
    c/omega_p, r = dx2/dx1 = 1, kappa = dx1/dt = 4, 8 particles per cell at the
    peak; to omega_p t = 450 (36000 steps).  The window moves with the beam at
    c; the beam centre sits at 0.6 n1 (the bunch, clipped at 4 sigma, fits with a margin)."""
    dx = (0.05, 0.05, 0.05)
    dt = dx[0] / 4.0
    sig = (1.0, 0.5, 0.5)
    n_peak = 100.0
    ppc_peak = 8.0
    vol = (2.0 * math.pi) ** 1.5 * sig[0] * sig[1] * sig[2]
    dV = dx[0] * dx[1] * dx[2]
    npart = int(round(n_peak * vol / (n_peak * dV / ppc_peak)))
    return Workload("drift-3d", 3, tuple(n), dx, dt, True, "yee", 36000,
                    {"npart": npart, "center": (0.6 * n[0], n[1] / 2, n[2] / 2), "sigma_phys": sig,
                     "gamma": 1000.0 / 0.51099895, "espread": 0.0, "divergence": 0.0, "n_peak": n_peak})


def transverse_partners(seed, cell, off, u, n):
    """One partner per particle at the same x1, at a uniform random position
    over the periodic transverse grid, with the same momentum: given the
    opposite charge and no force (a ballistic species), the partners cancel
    the transversely uniform part of every x1 slice's charge and current,
    which a periodic transverse grid would otherwise turn into a sheet field
    that open space does not have."""
    rng = np.random.default_rng(seed)
    X = cell + off
    for d in range(1, X.shape[1]):
        X[:, d] = rng.uniform(-0.5, n[d] - 0.5, X.shape[0])
    c, o = split_positions(X)
    return c, o, np.array(u, dtype=np.float64, copy=True)
