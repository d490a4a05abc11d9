"""Field loss around a moving bunch and its finite-difference gradient with
respect to the axial coefficients (TEST INFRASTRUCTURE ONLY).

The loss is written out from its definition on the FP64 oracle's fields:
  l_n = dx1 dx2 dt * [ sum over E1 points outside the box of E1^2
                       + sum over E2 points outside the box of (E2 - B3c)^2 ]
with E1 at ((i1 + 1/2) dx1, i2 dx2), E2 at (i1 dx1, (i2 + 1/2) dx2), B3c the
mean of B3 at i1 - 1/2 and i1 + 1/2 (same i2 + 1/2), all at integer time n,
and the box of step n centred at (x1 + v1 n dt, x2) with half-widths
(half1, half2).  L = sum over n = 1..N of l_n.  The transverse force on a
particle moving at c along x1 is q (E2 - B3); the bunch's own continuum field
makes it vanish, so outside the bunch it measures the numerical error the
paper attributes to the operators (Sec. 3).  The gradient is the plain
central difference of L in each coefficient.
"""
import numpy as np

from .pic import OracleSim


def outside(box, x1, x2, n, dt):
    c1 = box["x1"] + box["v1"] * n * dt
    return (np.abs(x1 - c1) > box["half1"]) | (np.abs(x2 - box["x2"]) > box["half2"])


def step_loss(E1, E2, B3, n, box, dx, dt):
    """l_n from E^n and B^n arrays of shape (n2, n1)."""
    n2, n1 = E1.shape
    i1 = np.arange(n1)[None, :]
    i2 = np.arange(n2)[:, None]
    m1 = outside(box, (i1 + 0.5) * dx[0], i2 * dx[1], n, dt)
    m2 = outside(box, i1 * dx[0], (i2 + 0.5) * dx[1], n, dt)
    B3c = 0.5 * (np.roll(B3, 1, axis=1) + B3)  # B3c(i1) = (B3(i1 - 1/2) + B3(i1 + 1/2)) / 2
    r = E2 - B3c
    return dx[0] * dx[1] * dt * (np.sum(np.where(m1, E1 * E1, 0.0)) + np.sum(np.where(m2, r * r, 0.0)))


def total_loss(w, C):
    """L for workload w (a dict with grid, particles, Q, box, nsteps) and coefficients C."""
    g = w["grid"]
    n, dx = g["n"][:2], g["dx"][:2]
    o = OracleSim(n, dx, g["dt"], C=list(C), window=False)
    o.add_particles(w["cell"].astype(np.float64) + w["offset"], w["u"], w["Q"], 0.0)
    L = 0.0
    for step in range(1, w["nsteps"] + 1):
        o.step(1)
        L += step_loss(o.field("E1"), o.field("E2"), o.field("B3"), step, w["box"], dx, g["dt"])
    o.close()
    return L


def fd_gradient(w, C, h=1e-4):
    """central differences (L(C + h e_l) - L(C - h e_l)) / 2h"""
    C = np.asarray(C, dtype=np.float64)
    g = np.zeros(C.size)
    for l in range(C.size):
        cp, cm = C.copy(), C.copy()
        cp[l] += h
        cm[l] -= h
        g[l] = (total_loss(w, cp) - total_loss(w, cm)) / (2 * h)
    return g
