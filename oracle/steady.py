"""Steady-state lattice fields of charges streaming along x1 on a periodic 2D
grid (TEST INFRASTRUCTURE ONLY).

Sec. 2.1 writes the fields of a particle moving only along x1 in terms of its
charge density: Fourier transforming the discrete Faraday and Ampere laws
(the operators acting on E and on B may differ), using Gauss's law and the
continuity equation J1 = [omega]_t rho / [k]_B1, gives

  E1 = -(i/[k]_B1) ([w]^2 - [k]_E1[k]_B1) / D rho,   E2 = i [k]_E2 / D rho,
  B3 = i ([k]_E2/[k]_B1) [w] / D rho,   D = [w]^2 - [k]_E1[k]_B1 - [k]_E2[k]_B2.

Here the grid is periodic and finite, so every wavenumber is a lattice one
and no integral or pole prescription is involved: a particle that advances
s cells every P steps deposits a density whose lattice transform at step n
is a sum of P frequencies omega_c dt = (k1 s dx1 + 2 pi c)/P, c = 0..P-1
(the aliased zones of App. A folded onto the time lattice).  Each frequency
gets the response above, with [w] = sin(omega dt/2)/(dt/2).  The result is
an exact time-periodic solution of the discrete equations that the PIC step
must carry forward unchanged, which is what the tests check.

Conventions are those of the PIC oracle: E1 at (i1+1/2, i2), E2 at
(i1, i2+1/2), B3 at (i1+1/2, i2+1/2), rho at nodes; E and rho at integer
steps, B and J at half steps, and B at integer step n reported as the mean of
B^{n-1/2} and B^{n+1/2} (the oracle's stored B).  Axial operators:
d+ (E -> B) with coefficients CE, d- (B -> E) with CB; Yee transverse.

Two modes have no frequency to divide by: the uniform mode (k = 0), where a
net current makes E1 grow linearly in time (-J_mean t, reported as such), and
the x1-uniform modes (k1 = 0, k2 != 0), which are static: B3 from the line
currents (Ampere with d_t E1 = 0), E2 from Gauss's law, E1 zero.
"""
import math

import numpy as np


def spline2(d):
    """Quadratic B-spline of a distance in cells."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    out = np.where(d <= 0.5, 0.75 - d * d, 0.0)
    mid = (d > 0.5) & (d < 1.5)
    return np.where(mid, 0.5 * (1.5 - d) ** 2, out)


def node_density(n1, n2, dx1, dx2, x1, x2, Q):
    """rho at the nodes of a periodic grid: Q S(i1 - x1) S(i2 - x2) / dV."""
    rho = np.zeros((n2, n1))
    c1, c2 = int(math.floor(x1 + 0.5)), int(math.floor(x2 + 0.5))
    for b in range(-2, 3):
        w2 = float(spline2(c2 + b - x2))
        for a in range(-2, 3):
            w1 = float(spline2(c1 + a - x1))
            rho[(c2 + b) % n2, (c1 + a) % n1] += Q * w1 * w2 / (dx1 * dx2)
    return rho


def axial_symbol(C, k1, dx1):
    """[k]_1 = sum_l C_l sin((2l-1) k1 dx1/2) / (dx1/2)  (App. C)."""
    s = np.zeros_like(k1)
    for l, c in enumerate(C, start=1):
        s = s + c * np.sin((2 * l - 1) * 0.5 * k1 * dx1)
    return s / (0.5 * dx1)


class SteadyState:
    """Fields of ballistic charges moving along x1 on an n1 x n2 periodic grid.

    particles: list of (x1, x2, Q, v) with positions in cells at step 0 and v
    the velocity in units of c.  Every particle must advance a whole number s
    of cells in P steps: v dt / dx1 = s / P (P is found from v_cells_per_step
    given as a fraction (s, P)).
    """

    def __init__(self, n, dx, dt, particles, step_fraction, CE=(1.0,), CB=None):
        self.n1, self.n2 = n
        self.dx1, self.dx2 = dx
        self.dt = dt
        s, P = step_fraction
        self.P = int(P)
        self.parts = []
        for (x1, x2, Q, v) in particles:
            sc = v * dt / self.dx1 * self.P
            sp = int(round(sc))
            if abs(sc - sp) > 1e-12:
                raise ValueError("particle must advance a whole number of cells every P steps")
            self.parts.append((float(x1), float(x2), float(Q), float(v), sp))
        CB = CE if CB is None else CB
        k1 = 2.0 * np.pi * np.fft.fftfreq(self.n1) / self.dx1
        k2 = 2.0 * np.pi * np.fft.fftfreq(self.n2) / self.dx2
        self.k1, self.k2 = k1, k2
        self.sE = axial_symbol(CE, k1, self.dx1)[None, :]
        self.sB = axial_symbol(CB, k1, self.dx1)[None, :]
        self.s2 = (np.sin(0.5 * k2 * self.dx2) / (0.5 * self.dx2))[:, None]
        self._modes = [self._particle_modes(p) for p in self.parts]

    def _particle_modes(self, part):
        """Frequencies and density amplitudes of one particle: rho_hat at
        step n = sum_c a_c exp(-i w_c n dt)."""
        x1, x2, Q, v, sp = part
        P = self.P
        dens = []
        for n in range(P):
            dens.append(np.fft.fft2(node_density(self.n1, self.n2, self.dx1, self.dx2,
                                                 x1 + n * v * self.dt / self.dx1, x2, Q)))
        dens = np.array(dens)  # [P, n2, n1]
        wdt = []
        amps = []
        for c in range(P):
            w = (self.k1 * self.dx1 * sp + 2.0 * np.pi * c) / P  # omega_c dt, per k1
            w = np.broadcast_to(w[None, :], (self.n2, self.n1))
            a = np.zeros((self.n2, self.n1), dtype=complex)
            for n in range(P):
                a += dens[n] * np.exp(1j * w * n)
            amps.append(a / P)
            wdt.append(w)
        return wdt, amps, v

    def fields(self, step):
        """E1, E2, B3 (arrays [i2][i1]) at integer step `step`."""
        dt = self.dt
        ph1 = np.exp(0.5j * self.k1 * self.dx1)[None, :]   # E1, B3 sit at i1 + 1/2
        ph2 = np.exp(0.5j * self.k2 * self.dx2)[:, None]   # E2, B3 sit at i2 + 1/2
        k1zero = (np.abs(self.k1) == 0.0)[None, :] & np.ones((self.n2, 1), dtype=bool)
        k2zero = (np.abs(self.k2) == 0.0)[:, None] & np.ones((1, self.n1), dtype=bool)
        E1h = np.zeros((self.n2, self.n1), dtype=complex)
        E2h = np.zeros_like(E1h)
        B3h = np.zeros_like(E1h)
        uniform_e1 = 0.0
        for (wdt, amps, v) in self._modes:
            for w, a in zip(wdt, amps):
                tw = np.sin(0.5 * w) / (0.5 * dt)            # [omega]_t
                D = tw * tw - self.sE * self.sB - self.s2 * self.s2
                rot = np.exp(-1j * w * step)                 # time dependence at step n
                with np.errstate(divide="ignore", invalid="ignore"):
                    dyn = ~k1zero
                    J1 = np.where(dyn, tw * a / self.sB, 0.0)
                    B3 = np.where(dyn, 1j * self.s2 * J1 / D, 0.0)
                    E1 = np.where(dyn, (-self.s2 * B3 - 1j * J1) / tw, 0.0)
                    E2 = np.where(dyn, self.sB * B3 / tw, 0.0)
                    # x1-uniform, x2-varying modes: static (only c with w = 0 carries them)
                    stat = k1zero & ~k2zero & (np.abs(w) < 1e-14)
                    Jl = v * a                               # line current of the x1-uniform density
                    B3 = np.where(stat, -1j * Jl / self.s2, B3)
                    E2 = np.where(stat, -1j * a / self.s2, E2)
                # B at integer steps: mean of the two half steps around it
                E1h += E1 * rot
                E2h += E2 * rot
                B3h += B3 * rot * np.cos(0.5 * w)
                uniform = k1zero & k2zero & (np.abs(w) < 1e-14)
                uniform_e1 += float(np.real((v * a)[uniform].sum()))
        E1 = np.fft.ifft2(E1h * ph1).real
        E2 = np.fft.ifft2(E2h * ph2).real
        B3 = np.fft.ifft2(B3h * ph1 * ph2).real
        # net current: d_t E1 = -J_mean for the uniform mode
        E1 += -uniform_e1 / (self.n1 * self.n2) * step * dt
        return E1, E2, B3

    def min_denominator(self):
        """Smallest |D| over the driven modes relative to (2/dx1)^2 (how close
        the finite grid comes to a resonance)."""
        best = np.inf
        for (wdt, amps, v) in self._modes:
            for w, a in zip(wdt, amps):
                tw = np.sin(0.5 * w) / (0.5 * self.dt)
                D = tw * tw - self.sE * self.sB - self.s2 * self.s2
                mask = (np.abs(a) > 1e-14 * np.abs(a).max()) & (np.abs(self.k1) > 0)[None, :]
                if mask.any():
                    best = min(best, float(np.abs(D[mask]).min()))
        return best * (0.5 * self.dx1) ** 2
