"""GPU parity of the current filter (the 5-pass filter with which Secs.
2.2-3 quote the filtered self-force; reading: four binomial passes and the
compensator c = 5 along x1, applied to J after the J1 correction): the HIP
path against the FP64 oracle with the same filter, element by element (FP64
within 1e-12, FP32 within 1e-5 of each component), with Yee and with the
customized solver, on a periodic x1 line (a box that covers the whole line
and one that does not) and in the 3D moving window with the fused and the
separate field updates; Gauss's law for the filtered density; the GPU's own
filtered Yee self-force against the k-space integral with the filter's
symbol; argument checks."""
import numpy as np
import pytest

from oracle import kspace
from oracle.fit import TABLE1
from oracle.pic import OracleSim
from tests.gpu_common import beam_species, field_errors, log, make_pair, particle_errors

pytestmark = pytest.mark.gpu

FIVE_PASS = (4, 5.0)


def _filtered_pair(ndim, n, dx, dt, C, window, sp, precision, fused=None):
    g, o, ids = make_pair(ndim, n, dx, dt, C, window, [sp], precision)
    g.set_current_filter(*FIVE_PASS)
    o.set_filter(*FIVE_PASS)
    if fused is not None:
        assert g.set_fused_fields(fused) == fused
    return g, o, ids[0]


def _ptol(precision):
    return 1e-12 if precision == "fp64" else 2e-5


@pytest.mark.parametrize("solver", ["yee", "custom"])
@pytest.mark.parametrize("n1,sigma1", [(128, 6.0), (32, 3.0)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_filter_2d_periodic_beam(solver, n1, sigma1, precision, tol):
    C = TABLE1 if solver == "custom" else (1.0,)
    n, dx, dt = (n1, 32), (1.0, 1.0), 0.25
    npart = 300
    sp = beam_species(7, npart, n, dx, 20.0, Q=-0.05, sigma_cells=(sigma1, 2.0), divergence=0.05, espread=0.05)
    g, o, sid = _filtered_pair(2, n, dx, dt, C, False, sp, precision)
    rho0 = g.diagnostics()
    g.profile_enable(True)
    g.step(60)
    o.step(60)
    prof = g.profile_read()
    assert prof["filter"][0] == 60, prof
    errs = field_errors(g, o)
    log("filter 2D %s n1=%d %s: %s" % (solver, n1, precision, errs))
    assert max(errs.values()) < tol, errs
    dxp, dup = particle_errors(g, o, sid, npart)
    assert dxp < _ptol(precision) and dup < _ptol(precision)
    # fields start at zero, so div E - F rho = -F rho(0) from then on: the
    # diagnostic's residual keeps the filtered density's initial maximum
    d = g.diagnostics()
    assert abs(d["gauss_max"] - rho0["gauss_max"]) < (1e-9 if precision == "fp64" else 1e-4) * rho0["gauss_max"]
    g.sync()


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_filter_3d_window_beam(fused, precision, tol):
    n, dx, dt = (72, 16, 16), (0.02, 0.05, 0.05), 0.005
    npart = 2000
    sp = beam_species(3, npart, n, dx, 1e4, Q=-1e-3, sigma_cells=(5.0, 1.0, 1.0), center_frac=0.6)
    g, o, sid = _filtered_pair(3, n, dx, dt, TABLE1, True, sp, precision, fused=fused)
    for k in (17, 1, 23):  # 41 steps in three calls, ten window shifts
        g.step(k)
        o.step(k)
    errs = field_errors(g, o)
    log("filter 3D fused=%s %s: %s" % (fused, precision, errs))
    assert max(errs.values()) < tol, errs
    dxp, dup = particle_errors(g, o, sid, npart)
    assert dxp < _ptol(precision) and dup < _ptol(precision)
    g.sync()


def test_filter_at_the_window_front():
    # a beam whose current reaches the window's leading cells: the passes
    # are cut off at the window's end as in the oracle
    n, dx, dt = (64, 24), (1.0, 1.0), 0.25
    sp = beam_species(5, 200, n, dx, 50.0, Q=-0.05, sigma_cells=(2.0, 2.0), center_frac=0.85)
    g, o, sid = _filtered_pair(2, n, dx, dt, TABLE1, True, sp, "fp64")
    g.step(12)
    o.step(12)
    errs = field_errors(g, o)
    log("filter at window front: %s" % errs)
    assert max(errs.values()) < 1e-12, errs
    g.sync()


def _filtered_window_self_force(n2, steps):
    from paper_1910_13529_amd.relpic import Sim
    grid = dict(ndim=2, n=(64, n2, 1), dx=(1.0, 1.0, 1.0), dt=0.25, window=True, window_speed=1.0)
    g = Sim(grid, precision="fp64")
    g.set_current_filter(*FIVE_PASS)
    sid = g.add_species(0.0, 1.0, 1)
    g.load_particles(sid, np.array([[32, n2 // 2]], dtype=np.int32), np.zeros((1, 2)), np.array([[1e8, 0.0, 0.0]]))
    g.step(steps)
    F1 = float(g.gather_particles(sid)[0, 0])
    g.close()
    return F1


def test_gpu_filtered_yee_self_force_matches_kspace_integral():
    # the oracle pin's extrapolation over the transverse width, on the HIP path
    f = {}
    for n2, steps in ((32, 1200), (64, 2400), (128, 8000)):
        log("filtered self-force: n2 = %d" % n2)
        f[n2] = _filtered_window_self_force(n2, steps)
    F_inf = (8.0 * f[128] - 6.0 * f[64] + f[32]) / 3.0
    F_th = kspace.KSpace("yee", 4.0, 1.0, order=2, beta=1.0, tpow=2, nus=tuple(range(-3, 4)),
                         filt=FIVE_PASS).lattice_self_force()
    log("filtered self-force: %s, extrapolated %.7f, k-space %.7f" % (f, F_inf, F_th))
    assert abs(F_inf - F_th) < 1e-3 * abs(F_th), (f, F_inf, F_th)


def test_filter_arguments():
    from paper_1910_13529_amd.relpic import RelpicError, Sim
    g = Sim(dict(ndim=2, n=(64, 16, 1), dx=(1.0, 1.0, 1.0), dt=0.25), precision="fp64")
    for bad in ((-1, 5.0), (17, 5.0), (4, float("inf")), (4, float("nan"))):
        with pytest.raises(RelpicError):
            g.set_current_filter(*bad)
    g.set_current_filter(0, float("nan"))  # off: c unused
    g.close()
    g = Sim(dict(ndim=2, n=(4100, 4, 1), dx=(1.0, 1.0, 1.0), dt=0.25), precision="fp32")
    with pytest.raises(RelpicError):
        g.set_current_filter(*FIVE_PASS)
    g.set_current_filter(0, 0.0)
    g.close()
