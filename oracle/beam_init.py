"""Self-consistent initial fields of charges streaming along x1 at beta -> 1
(TEST INFRASTRUCTURE ONLY).

Sec. 2.1 gives the fields of a charge moving along x1 in terms of its
density: E2 = i [k]_E2 rho / D, B3 = i ([k]_E2/[k]_B1) [w]_t rho / D,
D = [w]_t^2 - [k]_E.[k]_B.  When the axial operators satisfy
[k]_E1 [k]_B1 = [beta k1]_t^2 (the paper's [k]_1 = [k1]_t at beta = 1),
D = -[k]_perp^2 and each x1 slice carries the lattice transverse Poisson
field of its charge: -lap_perp phi = rho (Yee x2/x3 differences, periodic),
E_perp = -grad_perp phi, E1 = -(1 - beta^2) d1 phi, and B = beta x E on B's
lattice points (B3 at i1 + 1/2 is beta times the mean of E2 at i1 and
i1 + 1; B2 = -beta E3 likewise).  The part of a slice's charge that is
uniform over the transverse plane has no transverse field and is dropped.
Written here with numpy's FFT over each slice.
"""
import numpy as np


def beam_fields(rho, dx, beta, window=False):
    """rho: node charge density [i3][i2][i1] (3D) or [i2][i1] (2D), window-
    relative along x1.  Returns dict E1..B3 of the same shape."""
    rho = np.asarray(rho, dtype=np.float64)
    ndim = rho.ndim
    taxes = tuple(range(ndim - 1))            # transverse numpy axes (x3, x2 or x2)
    n_t = [rho.shape[a] for a in taxes]       # sizes along those axes
    dx_t = [dx[ndim - 1 - a] for a in taxes]  # their spacings (numpy axis a <-> dimension ndim-1-a)
    rh = np.fft.fftn(rho, axes=taxes)
    den = np.zeros(rh.shape[:-1])
    for a, (n, d) in enumerate(zip(n_t, dx_t)):
        s = 2.0 * np.sin(np.pi * np.arange(n) / n) / d
        shp = [1] * (ndim - 1)
        shp[a] = n
        den = den + (s ** 2).reshape(shp)
    with np.errstate(divide="ignore", invalid="ignore"):
        ph = np.where(den[..., None] > 0, rh / den[..., None], 0.0)
    phi = np.real(np.fft.ifftn(ph, axes=taxes))

    def nxt(f, axis):
        return np.roll(f, -1, axis=axis)

    def nxt1(f):
        # x1 neighbour: periodic, or zero beyond the window
        g = np.roll(f, -1, axis=-1)
        if window:
            g[..., -1] = 0.0
        return g

    out = {}
    x2ax = ndim - 2  # numpy axis of x2
    E2 = -(nxt(phi, x2ax) - phi) / dx[1]
    E3 = -(nxt(phi, 0) - phi) / dx[2] if ndim == 3 else np.zeros_like(phi)
    out["E1"] = -(1.0 - beta * beta) * (nxt1(phi) - phi) / dx[0]
    out["E2"] = E2
    out["E3"] = E3
    out["B1"] = np.zeros_like(phi)
    out["B2"] = -beta * 0.5 * (E3 + nxt1(E3))
    out["B3"] = beta * 0.5 * (E2 + nxt1(E2))
    return out


def init_oracle(sim, beta):
    """Set the oracle simulation's E and B to the self-consistent fields of its
    particles' charge (its own node density at the current positions)."""
    f = beam_fields(sim.rho(), sim.dx, beta, window=getattr(sim, "window", False))
    for nm, arr in f.items():
        sim.set_field(nm, arr)
    return f
