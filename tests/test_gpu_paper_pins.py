"""GPU runs of the paper-level pins, through the C ABI:

* the lattice steady state of a charge streaming along x1 (the Sec. 2.1
  response in terms of the density) is carried by the HIP step as by the
  oracle: FP64 within 1e-12, FP32 within 1e-5 of each component's maximum;
* the self-force diagnostic (relpic_gather_particles) and the line-out
  against the k-space field (relpic_e1_residual) match the oracle's gather
  and line-out element by element, and the k-space side matches the
  oracle's quadrature;
* the GPU's own Yee self-force, extrapolated over the transverse width as in
  the oracle pin, reproduces the k-space F1 with the PIC's gather (Eq. 19);
* in 3D the line-out matches the oracle's field and its k-space side the 3D
  k-space oracle.
"""
import math

import numpy as np
import pytest

from oracle import kspace
from oracle.fit import TABLE1
from oracle.pic import OracleSim
from oracle.steady import SteadyState
from tests.gpu_common import log

pytestmark = pytest.mark.gpu


def _split(x):
    c = np.floor(np.asarray(x, dtype=np.float64) + 0.5)
    return c.astype(np.int32), np.asarray(x, dtype=np.float64) - c


STEADY = [
    ("yee", (1.0, 1.0), [(20.0, 16.0, 1.0, 1.0)], (1, 4), 40),
    ("custom", (1.0, 1.0), [(20.0, 16.0, 1.0, 1.0)], (1, 4), 40),
    ("yee", (1.0, 1.5), [(20.25, 8.0, 1.0, 0.75), (40.0, 20.5, -0.5, -0.5)], (3, 16), 48),
    ("custom", (1.0, 1.5), [(20.25, 8.0, 1.0, 0.75), (40.0, 20.5, -0.5, -0.5)], (3, 16), 48),
]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("solver,dx,parts,frac,steps", STEADY)
def test_gpu_carries_the_lattice_steady_state(solver, dx, parts, frac, steps, precision, tol):
    from paper_1910_13529_amd.relpic import Sim
    n, dt = (64, 32), 0.25
    C = (1.0,) if solver == "yee" else tuple(TABLE1)
    log("steady state %s %s dx=%s, %d charges" % (solver, precision, dx, len(parts)))
    ss = SteadyState(n, dx, dt, parts, frac, CE=C)
    grid = dict(ndim=2, n=(n[0], n[1], 1), dx=(dx[0], dx[1], 1.0), dt=dt)
    g = Sim(grid, C=list(C) if len(C) > 1 else None, precision=precision)
    E1, E2, B3 = ss.fields(0)
    g.set_field("E1", E1)
    g.set_field("E2", E2)
    g.set_field("B3", B3)
    for (x1, x2, Q, v) in parts:
        u1 = math.copysign(1e8, v) if abs(v) == 1.0 else v / math.sqrt(1.0 - v * v)
        cell, off = _split([[x1, x2]])
        sid = g.add_species(0.0, Q, 1)
        g.load_particles(sid, cell, off, np.array([[u1, 0.0, 0.0]]))
    done = 0
    for k in (1, 3, 8, steps):  # several calls: the state carried across relpic_step calls
        g.step(k - done)
        done = k
        ref = ss.fields(k)
        for nm, r in zip(("E1", "E2", "B3"), ref):
            err = float(np.abs(g.field(nm) - r).max() / np.abs(r).max())
            assert err < tol, (nm, k, err)
    g.sync()


def _window_pair(n2, steps, precision):
    """GPU and oracle: a beta -> 1 unit charge on a node in a 64-cell window at
    c, Yee, kappa = 4, r = 1, ballistic."""
    from paper_1910_13529_amd.relpic import Sim
    grid = dict(ndim=2, n=(64, n2, 1), dx=(1.0, 1.0, 1.0), dt=0.25, window=True, window_speed=1.0)
    g = Sim(grid, precision=precision)
    sid = g.add_species(0.0, 1.0, 1)
    g.load_particles(sid, np.array([[32, n2 // 2]], dtype=np.int32), np.zeros((1, 2)), np.array([[1e8, 0.0, 0.0]]))
    g.step(steps)
    return g, sid


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_gpu_self_force_and_e1_residual_match_oracle(precision, tol):
    n2, steps = 32, 1200
    log("self-force diagnostic %s: n2 = %d, %d steps" % (precision, n2, steps))
    g, sid = _window_pair(n2, steps, precision)
    o = OracleSim((64, n2), (1.0, 1.0), 0.25, window=True, vwin=1.0)
    o.add_particles(np.array([[32.0, n2 / 2]]), np.array([[1e8, 0.0, 0.0]]), 1.0, 0.0)
    o.step(steps)
    x, _, _ = o.particles()
    EBo = o.gather_at(x[:1])[0]
    EBg = g.gather_particles(sid)[0]
    scale = np.abs(EBo).max()
    assert np.abs(EBg - EBo).max() < tol * scale, (EBg, EBo)
    # the line-out around the charge and the k-space field at the same points
    rel = np.arange(-12, 6)
    sim, th = g.e1_residual(sid, 0, rel, beta=1.0, shape_order=2, tpow=1, nu_max=3)
    ip = int(round(x[0, 0])) - o.window_start
    line = o.field("E1")[n2 // 2, ip + rel]
    assert np.abs(sim - line).max() < tol * np.abs(line).max()
    ks = kspace.KSpace("yee", 4.0, 1.0, order=2, beta=1.0, tpow=1, nus=tuple(range(-3, 4)))
    assert np.abs(th - ks.e1(rel)).max() < 1e-7 * np.abs(th).max()
    # next to the charge the residual is the transverse-size offset that the
    # oracle pin extrapolates away (far behind it the periodic x2 images'
    # wakes take over)
    near = (rel >= -2) & (rel <= 2)
    assert np.abs(sim - th)[near].max() < 0.1 * np.abs(th).max()
    g.sync()


def test_gpu_yee_self_force_matches_kspace_integral():
    # same extrapolation as the oracle pin, on the HIP path (FP64)
    f = {}
    for n2, steps in ((32, 1200), (64, 2400), (128, 8000)):
        log("self-force extrapolation: n2 = %d" % n2)
        g, sid = _window_pair(n2, steps, "fp64")
        f[n2] = float(g.gather_particles(sid)[0, 0])
        g.sync()
    F_inf = (8.0 * f[128] - 6.0 * f[64] + f[32]) / 3.0
    F_th = kspace.KSpace("yee", 4.0, 1.0, order=2, beta=1.0, tpow=2, nus=tuple(range(-3, 4))).lattice_self_force()
    assert abs(F_inf - F_th) < 1e-3 * abs(F_th), (f, F_inf, F_th)


def test_e1_residual_rejects_mismatched_theory():
    from paper_1910_13529_amd.relpic import RelpicError
    g, sid = _window_pair(32, 8, "fp64")
    with pytest.raises(RelpicError):
        g.e1_residual(sid, 0, [0, 1], kappa=3.0)  # not this run's kappa
    with pytest.raises(RelpicError):
        g.e1_residual(sid, 0, [0, 1], C=list(TABLE1))  # not this run's operator
    with pytest.raises(RelpicError):
        g.e1_residual(sid, 0, [-40])  # outside the window
    g.step(1)  # a quarter cell off the node
    with pytest.raises(RelpicError):
        g.e1_residual(sid, 0, [0])
    g.sync()


def test_gpu_e1_residual_3d_matches_oracle():
    # 3D: the line-out on the particle's row against the FP64 oracle's field,
    # and the theory side against the 3D k-space oracle (x3 closed form, x2
    # and k1 quadrature); Yee, kappa = 4, r2 = r3 = 1, a beta -> 1 charge on
    # a node after 40 steps (ten window shifts)
    from paper_1910_13529_amd.relpic import Sim
    n = (48, 16, 16)
    grid = dict(ndim=3, n=n, dx=(1.0, 1.0, 1.0), dt=0.25, window=True, window_speed=1.0)
    g = Sim(grid, precision="fp64")
    sid = g.add_species(0.0, 1.0, 1)
    g.load_particles(sid, np.array([[24, 8, 8]], dtype=np.int32), np.zeros((1, 3)), np.array([[1e8, 0.0, 0.0]]))
    g.step(40)
    o = OracleSim(n, (1.0, 1.0, 1.0), 0.25, window=True, vwin=1.0)
    o.add_particles(np.array([[24.0, 8.0, 8.0]]), np.array([[1e8, 0.0, 0.0]]), 1.0, 0.0)
    o.step(40)
    x, _, _ = o.particles()
    rel = np.array([-6, -3, -1, 0, 2], dtype=np.int32)
    sim, th = g.e1_residual(sid, 0, rel, beta=1.0, shape_order=2, tpow=1, nu_max=1)
    ip = int(round(x[0, 0])) - o.window_start
    line = o.field("E1")[8, 8, ip + rel]
    assert np.abs(sim - line).max() < 1e-12 * np.abs(line).max()
    k3 = kspace.KSpace3D("yee", 4.0, 1.0, 1.0, order=2, beta=1.0, tpow=1, nus=(-1, 0, 1))
    ref = np.array([k3.e1([v])[0] for v in rel])
    log("3D residual: sim %s theory %s oracle theory %s" % (sim, th, ref))
    assert np.abs(th - ref).max() < 1e-6 * np.abs(ref).max()
    g.close()
    o.close()
