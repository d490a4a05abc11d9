"""Pins of the operator variant of Sec. 3 with different axial operators on E
and on B, [k]_E1 != [k]_B1 with [k]_E1 [k]_B1 = [k1]_t^2.  With [k]_B1 the Yee
operator (the one Ampere's law, Gauss's law and the continuity equation use)
the Esirkepov current already conserves charge and no J1 correction is
needed; the fit of App. C then targets [k]_E1 = [k1]_t^2 / [k]_Yee."""
import math

import numpy as np
import pytest

from oracle import dispersion, fit, kspace
from oracle.pic import OracleSim
from oracle.steady import SteadyState

KAPPA = 4.0


def e_operator(M=16):
    return fit.fit_coefficients(KAPPA, M=M, target=lambda k: fit.target_e_with_yee_b(k, KAPPA))


def test_fit_of_the_e_operator_gives_the_time_operator_product():
    CE = e_operator()
    # first consistency row of App. C: the symbol's slope at k = 0 is 1
    assert abs(np.sum((2 * np.arange(1, 17) - 1) * CE) - 1.0) < 1e-12
    kh = np.linspace(1e-3, 1.0, 400)
    prod = fit.sym_custom(kh, CE) * fit.sym_yee(kh)
    tgt = fit.sym_time(kh, KAPPA) ** 2
    assert np.abs(prod / tgt - 1.0).max() < 1e-6
    # and is not the same-operator solution
    assert np.abs(CE - fit.TABLE1).max() > 1e-2


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("which", ["custom_e", "custom_b"])
def test_single_mode_dispersion_separate_operators(ndim, which):
    CE = tuple(e_operator())
    C, CB = (CE, (1.0,)) if which == "custom_e" else ((1.0,), CE)
    if ndim == 2:
        n, dx, m = (64, 48), (1.0, 1.2), (5, 3)
    else:
        n, dx, m = (48, 8, 40), (1.0, 1.1, 0.9), (4, 0, 2)
    dt = 0.25
    k = [2 * math.pi * m[d] / (n[d] * dx[d]) for d in range(ndim)]
    s = OracleSim(n, dx, dt, C=C, CB=CB, correct=False)
    idx = np.meshgrid(*[np.arange(n[d]) for d in reversed(range(ndim))], indexing="ij")
    pos = [idx[ndim - 1 - d] * dx[d] for d in range(ndim)]
    if ndim == 2:
        comp, phase, kk, dd = "E3", k[0] * pos[0] + k[1] * pos[1], (k[0], k[1]), (dx[0], dx[1])
    else:
        comp, phase, kk, dd = "E2", k[0] * pos[0] + k[2] * pos[2], (k[0], k[2]), (dx[0], dx[2])
    basis = np.cos(phase)
    s.set_field(comp, basis)
    w = dispersion.omega(kk, dd, dt, C1=C, CB1=CB)
    amps = []
    for it in range(41):
        amps.append((s.field(comp) * basis).sum() / (basis * basis).sum())
        s.field_only(1)
    nn = np.arange(len(amps))
    assert np.abs(np.array(amps) - np.cos(w * nn * dt)).max() < 1e-12
    # the product of the two symbols sets the frequency: swapping them changes nothing
    assert abs(w - dispersion.omega(kk, dd, dt, C1=CB, CB1=C)) < 1e-15
    assert abs(w - dispersion.omega(kk, dd, dt)) > 1e-4 * w  # and it is not Yee's


def _gauss_run(C, CB, correct=None, ndim=2, window=False):
    rng = np.random.default_rng(5)
    n, dx = ((64, 16), (1.0, 1.2)) if ndim == 2 else ((48, 10, 8), (1.0, 1.1, 0.9))
    s = OracleSim(n, dx, 0.25, C=C, CB=CB, correct=correct, window=window)
    lo, hi = (20, n[0] - 20) if window else (0, n[0])
    X = np.stack([rng.uniform(lo, hi, 40)] + [rng.uniform(0, n[d], 40) for d in range(1, ndim)], axis=1)
    u = rng.normal(0, 2.0, (40, 3))
    u[:, 0] += 3.0
    s.add_particles(X, u, -0.3, -1.0)
    r0 = s.div_e() - s.rho()
    scale = np.abs(s.rho()).max()
    s.step(12)
    return np.abs(s.div_e() - s.rho() - r0).max() / scale, s


@pytest.mark.parametrize("ndim", [2, 3])
def test_gauss_law_holds_without_correction_when_b_operator_is_yee(ndim):
    CE = tuple(e_operator())
    err, s = _gauss_run(CE, (1.0,), ndim=ndim)
    assert err < 1e-12
    assert np.abs(s.field("E1")).max() > 0
    # the same customized operator on both sides needs the correction: without it Gauss breaks
    err_nc, _ = _gauss_run(CE, CE, correct=False, ndim=ndim)
    assert err_nc > 1e-4
    # and a customized B operator with the correction holds again
    err_c, _ = _gauss_run((1.0,), CE, ndim=ndim)
    assert err_c < 1e-12


def test_window_variant_needs_no_correction_taps():
    CE = tuple(e_operator())
    s = OracleSim((96, 16), (1.0, 1.0), 0.25, C=CE, CB=(1.0,), window=True)
    assert s.correction_halfwidth == 0
    s2 = OracleSim((96, 16), (1.0, 1.0), 0.25, C=(1.0,), CB=CE, window=True)
    assert s2.correction_halfwidth > 20


@pytest.mark.parametrize("which", ["custom_e", "custom_b"])
def test_steady_state_carried_with_separate_operators(which):
    CE = tuple(e_operator())
    C, CB = (CE, (1.0,)) if which == "custom_e" else ((1.0,), CE)
    n, dx, dt = (64, 32), (1.0, 1.5), 0.25
    parts = [(20.25, 8.0, 1.0, 0.75), (40.0, 20.5, -0.5, -0.5)]
    ss = SteadyState(n, dx, dt, parts, (3, 16), CE=C, CB=CB)
    assert ss.min_denominator() > 1e-12
    o = OracleSim(n, dx, dt, C=C, CB=CB)
    for nm, f in zip(("E1", "E2", "B3"), ss.fields(0)):
        o.set_field(nm, f)
    for (x1, x2, Q, v) in parts:
        o.add_particles(np.array([[x1, x2]]), np.array([[v / math.sqrt(1 - v * v), 0.0, 0.0]]), Q, 0.0)
    for k in (1, 5, 48):
        o.step(k - o.steps_done)
        for nm, r in zip(("E1", "E2", "B3"), ss.fields(k)):
            assert np.abs(o.field(nm) - r).max() < 1e-12 * np.abs(r).max(), (nm, k)


def test_kspace_variant_has_no_fundamental_zone_cerenkov():
    # [k]_E1 [k]_B1 = [k1]_t^2: the denominator error of the nu1 = 0 zone
    # vanishes below khat = 1 as for [k]_E1 = [k]_B1 = [k1]_t (Table 2)
    CE = e_operator()
    ks = kspace.KSpace("custom", KAPPA, 1.0, order=2, C=CE, CB=[1.0], nus=(0,))
    kh = np.linspace(1e-3, 1.0, 2000)
    assert np.abs(ks.A(kh, 0)).max() < 1e-6
    assert kspace.regime_nu0(ks) in ("space-charge", "mixed")
    yee = kspace.KSpace("yee", KAPPA, 1.0, order=2, nus=(0,)).self_force()
    f = ks.self_force()
    assert abs(f) < 0.02 * abs(yee)
