"""Full-size checks at the 3D beam configuration (512 x 256 x 256 cells, 2^22
particles, FP32, customized solver of Table 1, fused field update: the launch
configuration the benchmark times), through properties that hold at any size
and do not need the oracle to run the whole grid:

* a discrete vacuum eigenmode advances as cos(omega n dt) with omega from the
  closed-form dispersion relation of the discrete operators (Eq. 4);
* particles without charge or force move ballistically: x^n = x^0 + n dt u / gamma
  in cell units, across window shifts and a re-sort;
* the charge-conserving deposit keeps div E - rho at its t = 0 value
  (fields start at zero, so the Gauss residual's maximum stays max |rho(0)|)
  and loses no charge."""
import math

import numpy as np
import pytest

from oracle import dispersion, fit
from paper_1910_13529_amd import inputs
from tests.gpu_common import log

pytestmark = pytest.mark.gpu

TABLE1 = tuple(fit.TABLE1)
N = (512, 256, 256)


def _sim(window):
    from paper_1910_13529_amd.relpic import Sim
    w = inputs.config_beam3d(n=N)
    grid = dict(ndim=3, n=w.n, dx=w.dx, dt=w.dt, window=window, window_speed=1.0)
    g = Sim(grid, C=list(TABLE1), precision="fp32")
    assert g.set_fused_fields(True)
    return g, w


def test_fullsize_vacuum_mode_fp32():
    g, w = _sim(False)
    m = (8, 0, 4)
    k1 = 2 * math.pi * m[0] / (N[0] * w.dx[0])
    k3 = 2 * math.pi * m[2] / (N[2] * w.dx[2])
    i3, _, i1 = np.meshgrid(np.arange(N[2]), np.arange(N[1]), np.arange(N[0]), indexing="ij", sparse=True)
    basis = np.cos(k1 * i1 * w.dx[0] + k3 * i3 * w.dx[2]) * np.ones((1, N[1], 1))
    g.set_field("E2", basis)
    om = dispersion.omega((k1, k3), (w.dx[0], w.dx[2]), w.dt, C1=TABLE1)
    norm = float((basis * basis).sum())
    done = 0
    for stop in (20, 45):
        g.step(stop - done)
        done = stop
        amp = float((g.field("E2") * basis).sum()) / norm
        log("full-size mode: step %d amplitude %.9f expected %.9f" % (stop, amp, math.cos(om * stop * w.dt)))
        assert abs(amp - math.cos(om * stop * w.dt)) < 2e-5
    g.close()


def test_fullsize_ballistic_beam_fp32():
    g, w = _sim(True)
    cell, off, u = inputs.beam_inputs(w, seed=2)
    n = len(cell)
    sid = g.add_species(0.0, 0.0, n)  # q/m = 0 and no charge: no force, no current
    g.load_particles(sid, cell, off, u)
    steps = 0
    for k in (1, 15, 25):  # ten window shifts, a re-sort after 25 steps
        g.step(k)
        steps += k
    c, o, uu, alive = g.particles(sid, n)
    assert alive.all()
    gam = np.sqrt(1.0 + (u * u).sum(axis=1))
    expect = cell + off + steps * w.dt * u / gam[:, None] / np.asarray(w.dx)[None, :]
    err = float(np.abs((c + o) - expect).max())
    log("full-size ballistic beam: %d particles, %d steps, max position error %.3g cells" % (n, steps, err))
    assert err < 1e-5
    assert float(np.abs(uu - u).max() / np.abs(u).max()) < 1e-7
    d = g.diagnostics()
    assert d["w_field"] == 0.0 and d["n_alive"] == n
    g.close()


def test_fullsize_beam_charge_conservation_fp32():
    g, w = _sim(True)
    cell, off, u = inputs.beam_inputs(w, seed=2)
    n = len(cell)
    sid = g.add_species(-1.0, inputs.beam_charge(w), n)
    g.load_particles(sid, cell, off, u)
    d0 = g.diagnostics()
    assert d0["rho_max"] > 0 and abs(d0["gauss_max"] - d0["rho_max"]) < 1e-12 * d0["rho_max"]
    g.step(30)  # seven window shifts, fused updates
    d = g.diagnostics()
    log("full-size beam: rho_max(0) %.9g gauss_max(30) %.9g charge %.12g -> %.12g" %
        (d0["rho_max"], d["gauss_max"], d0["charge"], d["charge"]))
    assert d["n_alive"] == n and d["error_word"] == 0
    assert abs(d["charge"] - d0["charge"]) < 1e-9 * abs(d0["charge"])
    assert abs(d["gauss_max"] - d0["rho_max"]) < 1e-5 * d0["rho_max"]
    g.close()
