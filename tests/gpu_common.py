"""Shared helpers for the GPU parity tests: build the same seeded run on the
HIP path (through the C ABI) and on the FP64 CPU oracle, and compare."""
import math
import sys

import numpy as np

from oracle.pic import OracleSim
from paper_1910_13529_amd import inputs


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_pair(ndim, n, dx, dt, C, window, species, precision="fp64"):
    """species: list of (Q, qm, cell, offset, u, capacity).  Returns (gpu, oracle, ids)."""
    from paper_1910_13529_amd.relpic import Sim
    grid = dict(ndim=ndim, n=tuple(n) + (1,) * (3 - ndim), dx=tuple(dx) + (1.0,) * (3 - ndim), dt=dt,
                window=window, window_speed=1.0)
    g = Sim(grid, C=list(C) if len(C) > 1 else None, precision=precision)
    o = OracleSim(n, dx, dt, C=C, window=window)
    ids = []
    for (Q, qm, cell, off, u, cap) in species:
        sid = g.add_species(qm, Q, cap)
        if len(cell):
            g.load_particles(sid, cell, off, u)
            o.add_particles(cell.astype(np.float64) + off, u, Q, qm)
        ids.append(sid)
    return g, o, ids


# a component whose oracle maximum is below this fraction of its field's
# (E or B) maximum is the small difference of large terms (B1 of an axial
# beam: the x2 and x3 curls of E2 and E3 nearly cancel); its rounding error
# is set by those terms, so it is held to its field's maximum instead of its
# own
CANCEL_FRACTION = 1e-2


def field_errors(g, o, names=("E1", "E2", "E3", "B1", "B2", "B3")):
    """Per component: max |f_gpu - f_oracle| / max |f_oracle| of that same
    component; a cancelling component (oracle maximum below CANCEL_FRACTION of
    its field's maximum) is divided by its field's maximum instead."""
    gv = {nm: g.field(nm) for nm in names}
    ov = {nm: o.field(nm) for nm in names}
    own = {nm: float(np.abs(ov[nm]).max()) for nm in names}
    group = {grp: max([own[nm] for nm in names if nm[0] == grp] or [0.0]) for grp in ("E", "B")}
    errs = {}
    for nm in names:
        d = float(np.abs(gv[nm] - ov[nm]).max())
        sc = own[nm] if own[nm] >= CANCEL_FRACTION * group[nm[0]] else group[nm[0]]
        errs[nm] = d / sc if sc > 0 else d
    return errs


def particle_errors(g, o, sid, n_expected):
    cell, off, u, alive = g.particles(sid, n_expected)
    xo, uo, ao = o.particles()
    assert len(alive) == len(ao)
    assert (alive == ao).all()
    xg = cell.astype(np.float64) + off
    dx = np.abs(xg[alive] - xo[ao]).max() if alive.any() else 0.0
    umag = np.maximum(np.linalg.norm(uo[ao], axis=1), 1e-300)
    du = (np.linalg.norm(u[alive] - uo[ao], axis=1) / umag).max() if alive.any() else 0.0
    return float(dx), float(du)


def beam_species(seed, npart, n, dx, gamma, Q=-1e-3, sigma_cells=(4.0, 1.0, 1.0), center_frac=0.6,
                 divergence=1e-3, espread=0.01):
    ndim = len(n)
    center = [center_frac * n[0]] + [n[d] / 2.0 for d in range(1, ndim)]
    cell, off, u = inputs.gaussian_bunch(seed, npart, center, sigma_cells[:ndim], gamma, espread, divergence,
                                         ndim=ndim, clip_sigmas=3.0)
    return (Q, -1.0, cell, off, u, npart)
