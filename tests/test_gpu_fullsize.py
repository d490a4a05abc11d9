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


@pytest.mark.parametrize("precision,utol,xtol", [("fp64", 1e-12, 1e-12), ("fp32", 2e-5, 1e-4)])
def test_fullsize_gather_push_sampled(precision, utol, xtol):
    # one push of the full beam on the full grid (periodic x1, the same kernels
    # as the moving window) against the oracle's gather and Boris push of 4096
    # sampled particles in the GPU's own fields E^n, B^n
    from oracle.pic import OracleSim, boris
    from paper_1910_13529_amd.relpic import Sim
    w = inputs.config_beam3d(n=N)
    g = Sim(dict(ndim=3, n=w.n, dx=w.dx, dt=w.dt, window=False), C=list(TABLE1), precision=precision)
    assert g.set_fused_fields(True)
    cell, off, u = inputs.beam_inputs(w, seed=2)
    n = len(cell)
    sid = g.add_species(-1.0, inputs.beam_charge(w), n)
    g.load_particles(sid, cell, off, u)
    g.step(10)
    fields = {nm: g.field(nm) for nm in ("E1", "E2", "E3", "B1", "B2", "B3")}
    c0, o0, u0, a0 = g.particles(sid, n)
    g.step(1)
    c1, o1, u1, a1 = g.particles(sid, n)
    g.close()
    o = OracleSim(N, w.dx, w.dt, C=TABLE1, window=False)
    for nm in list(fields):
        o.set_field(nm, fields.pop(nm))
    sel = np.random.default_rng(7).choice(np.flatnonzero(a0 & a1), 4096, replace=False)
    x0 = c0[sel] + o0[sel]
    EB = o.gather_at(x0)
    o.close()
    un = np.array([boris(-1.0, w.dt, EB[i], u0[p]) for i, p in enumerate(sel)])
    gam = np.sqrt(1.0 + (un * un).sum(axis=1))
    xn = x0 + w.dt * un / gam[:, None] / np.asarray(w.dx)[None, :]
    du = float((np.linalg.norm(u1[sel] - un, axis=1) / np.linalg.norm(un, axis=1)).max())
    d = (c1[sel] + o1[sel]) - xn
    nn = np.asarray(N, dtype=np.float64)[None, :]
    d = (d + nn / 2) % nn - nn / 2  # periodic wrap
    dx_max = float(np.abs(d).max())
    # the momentum change itself (|u| ~ 1e4 hides it in FP32 storage)
    kick = un - u0[sel]
    dkick = float(np.abs((u1[sel] - u0[sel]) - kick).max() / np.abs(kick).max())
    log("full-size sampled push %s: max |du|/|u| %.3g, max |dx| %.3g cells, kick error %.3g" %
        (precision, du, dx_max, dkick))
    assert du < utol and dx_max < xtol
    if precision == "fp64":
        assert dkick < 1e-11


def test_fullsize_beam_1000_steps_fp32():
    # the full run length of the 3D beam configuration (1000 steps, 250
    # window shifts, 40 re-sorts) in the benchmark's launch configuration:
    # no particle lost, charge conserved, the Gauss residual still at its
    # t = 0 value, finite energies
    g, w = _sim(True)
    cell, off, u = inputs.beam_inputs(w, seed=2)
    n = len(cell)
    sid = g.add_species(-1.0, inputs.beam_charge(w), n)
    g.load_particles(sid, cell, off, u)
    d0 = g.diagnostics()
    g.step(1000)
    d = g.diagnostics()
    log("full-size beam, 1000 steps: window start %d, alive %d, charge %.12g -> %.12g, gauss_max %.9g (rho_max(0) %.9g), "
        "w_field %.6g, w_kin %.9g -> %.9g" % (d["window_start"], d["n_alive"], d0["charge"], d["charge"], d["gauss_max"],
                                              d0["rho_max"], d["w_field"], d0["w_kin"], d["w_kin"]))
    assert d["step"] == 1000 and d["window_start"] == 250
    assert d["n_alive"] == n and d["error_word"] == 0
    assert abs(d["charge"] - d0["charge"]) < 1e-9 * abs(d0["charge"])
    assert abs(d["gauss_max"] - d0["rho_max"]) < 1e-4 * d0["rho_max"]
    assert math.isfinite(d["w_field"]) and d["w_field"] > 0
    # the bunch barely exchanges energy with its own fields at gamma = 1e4
    assert abs(d["w_kin"] - d0["w_kin"]) < 1e-3 * d0["w_kin"]
    g.close()
