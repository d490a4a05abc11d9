"""Pins of the self-consistent initial fields of a beam streaming along x1
(oracle/beam_init.py; Sec. 2.1's fields in terms of rho, ultra-relativistic
limit): Gauss's law in every slice, the transversely uniform mode dropped,
and a beam started in these fields keeping them (moving with it) under the
customized solver, where a start in zero fields does not."""
import numpy as np
import pytest

from oracle.beam_init import beam_fields, init_oracle
from oracle.fit import TABLE1
from oracle.pic import OracleSim
from paper_1910_13529_amd import inputs


def _beam(o, n, ndim, seed=3, npart=2000, neutralize=True, Q=-0.01):
    centre = (n[0] / 2,) + tuple(n[d] / 2 for d in range(1, ndim))
    sig = (8.0,) + (3.0,) * (ndim - 1)
    cell, off, u = inputs.gaussian_bunch(seed, npart, centre, sig, 10.0, ndim=ndim)
    x = cell + off
    u[:, 0] = 1e8  # u / gamma rounds to beta = 1
    u[:, 1:] = 0.0
    o.add_particles(x, u, Q, 0.0)
    if neutralize:
        # same x1 as each beam particle, uniform over the transverse plane,
        # opposite charge: every slice's transversely uniform charge cancels
        rng = np.random.default_rng(seed + 1)
        xn = x.copy()
        for d in range(1, ndim):
            xn[:, d] = rng.uniform(-0.5, n[d] - 0.5, len(x))
        o.add_particles(xn, u, -Q, 0.0)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("neutralize", [True, False])
def test_init_keeps_gauss_in_every_slice(ndim, neutralize):
    n = (64, 24, 20)[:ndim]
    dx = (1.0, 0.8, 1.1)[:ndim]
    o = OracleSim(n, dx, 0.2)
    _beam(o, n, ndim, npart=600, neutralize=neutralize)
    init_oracle(o, 1.0)
    rho = o.rho()
    taxes = tuple(range(ndim - 1))
    mean = rho.mean(axis=taxes, keepdims=True)
    res = o.div_e() - (rho - mean)
    assert np.abs(res).max() < 1e-12 * np.abs(rho).max()
    if neutralize:
        assert np.abs(mean).max() < 1e-13 * np.abs(rho).max()
    # B = beta x E on B's points: B3 is E2 moved half a cell along x1
    f = {nm: o.field(nm) for nm in ("E2", "B3", "E1", "B1")}
    assert np.abs(f["B3"] - 0.5 * (f["E2"] + np.roll(f["E2"], -1, axis=-1))).max() < 1e-15 * np.abs(f["E2"]).max()
    assert np.abs(f["E1"]).max() == 0.0 and np.abs(f["B1"]).max() == 0.0


def test_beam_keeps_its_initial_fields_with_the_customized_solver():
    n, steps = (128, 64), 40
    err = {}
    for solver, C in (("custom", tuple(TABLE1)), ("yee", (1.0,))):
        for init in (True, False):
            o = OracleSim(n, (1.0, 1.0), 0.25, C=C)
            _beam(o, n, 2)
            f0 = beam_fields(o.rho(), o.dx, 1.0)
            if init:
                init_oracle(o, 1.0)
            o.step(steps)  # beta = 1, dt = dx1/4: the beam moved 10 cells
            err[solver, init] = max(np.abs(o.field(nm) - np.roll(f0[nm], steps // 4, axis=-1)).max()
                                    for nm in ("E2", "B3")) / np.abs(f0["E2"]).max()
    # the customized solver carries the initial field along with the beam (a
    # few percent from the beam's shot noise in the aliased zones); a start in
    # zero fields is far from it, and so is Yee (its fundamental zone radiates)
    assert err["custom", True] < 0.1
    assert err["custom", False] > 0.5
    assert err["yee", True] > 2 * err["custom", True]
