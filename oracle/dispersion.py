"""Closed-form vacuum dispersion of the discrete Maxwell operators
(TEST INFRASTRUCTURE ONLY).

Eq. 4 with J = 0: a transverse vacuum eigenmode of wavevector k satisfies
[omega]_t^2 = [k]_E . [k]_B (the operators on E and on B may differ along x1,
Sec. 3), with the leapfrog time symbol
[omega]_t = sin(omega dt/2)/(dt/2).  For [k]_E = [k]_B this reads
  sin^2(omega dt/2) = (dt/2)^2 sum_d [k]_d^2,
[k]_d = sin(k_d dx_d/2)/(dx_d/2) (Yee, Eq. 14) and, along x1 for the
customized solver, sum_l C_l sin((2l-1) k1 dx1/2)/(dx1/2) (App. C).
"""
import math

import numpy as np


def k_symbol(k, dx, C=(1.0,)):
    acc = 0.0
    for l, c in enumerate(C, start=1):
        acc += c * math.sin((2 * l - 1) * k * dx / 2.0)
    return acc / (dx / 2.0)


def omega(kvec, dxvec, dt, C1=(1.0,), CB1=None):
    """Angular frequency of the eigenmode; C1 is the x1 stencil acting on E
    (and on B unless CB1 gives that one), Yee transverse: sin^2(omega dt/2)
    = (dt/2)^2 ([k]_E1 [k]_B1 + sum_d [k]_d^2)."""
    s = k_symbol(kvec[0], dxvec[0], C1) * k_symbol(kvec[0], dxvec[0], C1 if CB1 is None else CB1)
    for k, dx in zip(kvec[1:], dxvec[1:]):
        s += k_symbol(k, dx) ** 2
    if s < 0.0:
        raise ValueError("[k]_E1 [k]_B1 < 0: no real frequency")
    arg = (dt / 2.0) * math.sqrt(s)
    if arg >= 1.0:
        raise ValueError("unstable: (dt/2)|[k]| >= 1")
    return 2.0 / dt * math.asin(arg)


def courant_number(n, dxvec, dt, C1=(1.0,), CB1=None):
    """max over the grid's modes of (dt/2) sqrt([k]_E . [k]_B); the scheme is
    stable below 1."""
    s = 0.0
    kh = np.linspace(0.0, math.pi / 2.0, 4097)
    sym = np.zeros_like(kh)
    symb = np.zeros_like(kh)
    for l, c in enumerate(C1, start=1):
        sym += c * np.sin((2 * l - 1) * kh)
    for l, c in enumerate(C1 if CB1 is None else CB1, start=1):
        symb += c * np.sin((2 * l - 1) * kh)
    s += np.abs(sym * symb).max() / (dxvec[0] / 2.0) ** 2
    for dx in dxvec[1:]:
        s += (1.0 / (dx / 2.0)) ** 2
    return (dt / 2.0) * math.sqrt(s)
