"""GPU parity of the operator variant of Sec. 3 with different axial
operators on E and on B ([k]_E1 != [k]_B1, [k]_E1 [k]_B1 = [k1]_t^2): the
HIP path against the FP64 oracle run with the same two operators, element
by element (FP64 within 1e-12, FP32 within 1e-5 of each component), with Yee
on B (no J1 correction) and with the customized operator on B (correction
on), in 2D and in the 3D moving window with the fused and the separate
field updates; the closed-form dispersion of the product operator; the
lattice steady state; the k-space field with the two symbols."""
import math

import numpy as np
import pytest

from oracle import dispersion, fit, kspace
from oracle.pic import OracleSim
from oracle.steady import SteadyState
from paper_1910_13529_amd import inputs
from tests.gpu_common import beam_species, field_errors, log, particle_errors

pytestmark = pytest.mark.gpu


def _e_operator():
    return tuple(fit.fit_coefficients(4.0, M=16, target=lambda k: fit.target_e_with_yee_b(k, 4.0)))


def _ops(which):
    CE = _e_operator()
    return (CE, (1.0,)) if which == "yee_b" else ((1.0,), CE)


def _pair(ndim, n, dx, dt, C, CB, window, sp, precision, fused=None):
    from paper_1910_13529_amd.relpic import Sim
    grid = dict(ndim=ndim, n=tuple(n) + (1,) * (3 - ndim), dx=tuple(dx) + (1.0,) * (3 - ndim), dt=dt,
                window=window, window_speed=1.0)
    g = Sim(grid, C=list(C), CB=list(CB), precision=precision)
    if fused is not None:
        assert g.set_fused_fields(fused) == fused
    o = OracleSim(n, dx, dt, C=C, CB=CB, window=window)
    Q, qm, cell, off, u, cap = sp
    sid = g.add_species(qm, Q, cap)
    g.load_particles(sid, cell, off, u)
    o.add_particles(cell.astype(np.float64) + off, u, Q, qm)
    return g, o, sid


@pytest.mark.parametrize("which", ["yee_b", "custom_b"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_variant_2d_periodic_beam(which, precision, tol):
    C, CB = _ops(which)
    n, dx, dt = (128, 32), (1.0, 1.0), 0.25
    sp = beam_species(7, 300, n, dx, 20.0, Q=-0.05, sigma_cells=(6.0, 2.0), divergence=0.05, espread=0.05)
    g, o, sid = _pair(2, n, dx, dt, C, CB, False, sp, precision)
    assert (g.correction_halfwidth == 0) == (which == "yee_b")
    rho0 = g.diagnostics()["rho_max"]  # fields start at zero: div E - rho = -rho(0) from then on
    g.step(60)
    o.step(60)
    errs = field_errors(g, o)
    log("variant 2D %s %s: %s" % (which, precision, errs))
    assert max(errs.values()) < tol, errs
    dxp, dup = particle_errors(g, o, sid, 300)
    assert dxp < (1e-12 if precision == "fp64" else 2e-5) and dup < (1e-12 if precision == "fp64" else 2e-5)
    # Gauss's law with the divergence of the operator on B: the residual keeps its t = 0 value
    d = g.diagnostics()
    assert abs(d["gauss_max"] - rho0) < (1e-9 if precision == "fp64" else 1e-4) * rho0, (d, rho0)
    g.sync()


@pytest.mark.parametrize("which", ["yee_b", "custom_b"])
@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_variant_3d_window_beam(which, fused, precision, tol):
    C, CB = _ops(which)
    n, dx, dt = (72, 16, 16), (0.02, 0.05, 0.05), 0.005
    sp = beam_species(3, 2000, n, dx, 1e4, Q=-1e-3, sigma_cells=(5.0, 1.0, 1.0), center_frac=0.6)
    g, o, sid = _pair(3, n, dx, dt, C, CB, True, sp, precision, fused=fused)
    for k in (17, 1, 23):  # 41 steps in three calls, ten window shifts
        g.step(k)
        o.step(k)
    errs = field_errors(g, o)
    log("variant 3D %s fused=%s %s: %s" % (which, fused, precision, errs))
    assert max(errs.values()) < tol, errs
    dxp, dup = particle_errors(g, o, sid, 2000)
    assert dxp < (1e-12 if precision == "fp64" else 2e-5) and dup < (1e-12 if precision == "fp64" else 2e-5)
    g.sync()


def test_variant_dispersion_and_steady_state_fp64():
    from paper_1910_13529_amd.relpic import Sim
    C, CB = _ops("yee_b")
    # single vacuum mode: phase advance from sin^2(w dt/2) = (dt/2)^2 ([k]_E1 [k]_B1 + [k]_2^2)
    n, dx, dt, m = (64, 48), (1.0, 1.2), 0.25, (5, 3)
    grid = dict(ndim=2, n=(n[0], n[1], 1), dx=(dx[0], dx[1], 1.0), dt=dt)
    g = Sim(grid, C=list(C), CB=list(CB), precision="fp64")
    k = [2 * math.pi * m[d] / (n[d] * dx[d]) for d in range(2)]
    i2, i1 = np.meshgrid(np.arange(n[1]), np.arange(n[0]), indexing="ij")
    basis = np.cos(k[0] * i1 * dx[0] + k[1] * i2 * dx[1])
    g.set_field("E3", basis)
    w = dispersion.omega(k, dx, dt, C1=C, CB1=CB)
    for stop in (10, 40):
        g.step(stop - g.get_step()[0])
        amp = float((g.field("E3") * basis).sum() / (basis * basis).sum())
        assert abs(amp - math.cos(w * stop * dt)) < 1e-12, (stop, amp)
    g.close()
    # lattice steady state of two streaming charges
    n, dx = (64, 32), (1.0, 1.5)
    parts = [(20.25, 8.0, 1.0, 0.75), (40.0, 20.5, -0.5, -0.5)]
    ss = SteadyState(n, dx, dt, parts, (3, 16), CE=C, CB=CB)
    grid = dict(ndim=2, n=(n[0], n[1], 1), dx=(dx[0], dx[1], 1.0), dt=dt)
    g = Sim(grid, C=list(C), CB=list(CB), precision="fp64")
    for nm, f in zip(("E1", "E2", "B3"), ss.fields(0)):
        g.set_field(nm, f)
    for (x1, x2, Q, v) in parts:
        c = np.floor(np.array([[x1, x2]]) + 0.5)
        sid = g.add_species(0.0, Q, 1)
        g.load_particles(sid, c.astype(np.int32), np.array([[x1, x2]]) - c, np.array([[v / math.sqrt(1 - v * v), 0, 0]]))
    g.step(48)
    for nm, r in zip(("E1", "E2", "B3"), ss.fields(48)):
        assert np.abs(g.field(nm) - r).max() < 1e-12 * np.abs(r).max(), nm
    g.close()


def test_variant_kspace_matches_oracle():
    from paper_1910_13529_amd import relpic
    C, CB = _ops("yee_b")
    rel = np.arange(-6, 4)
    got = relpic.kspace_e1(rel, C=list(C), CB=list(CB), kappa=4.0, r=1.0, beta=1.0, order=2, tpow=1, nu_max=2)
    ref = kspace.KSpace("custom", 4.0, 1.0, order=2, beta=1.0, C=C, CB=CB, tpow=1, nus=(-2, -1, 0, 1, 2)).e1(rel)
    assert np.abs(got - ref).max() < 1e-7 * np.abs(ref).max()
