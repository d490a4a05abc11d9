"""Pins of the PIC oracle itself against what the paper fixes at the level of
a whole PIC run (not only of its k-space formulas):

* the field gather: every staggered component is interpolated from its own
  lattice points with the quadratic B-spline, which reproduces a quadratic
  field in closed form (x^2 + 1/4: the spline's variance);
* the steady state of Sec. 2.1: the discrete Maxwell equations with the
  continuity equation give the fields of a charge streaming along x1 in
  terms of its density (E1, E2, B3 through [omega]_t and the operators'
  symbols); on a periodic grid this is an exact time-periodic lattice
  solution, and the PIC step started from it must carry it unchanged;
* the self-force of Sec. 2.2 (Eq. 19): a beta -> 1 charge on the Yee grid at
  kappa = 4, r = 1 measures, extrapolated to an unbounded transverse grid,
  the F1 of the k-space integral (Eq. 13) with the PIC's own gather;
* Table 2: the Yee solver's fundamental zone radiates (a steady Cerenkov
  drag, so the field energy grows at a constant rate) while the customized
  solver's does not.
"""
import math

import numpy as np
import pytest

from oracle import kspace
from oracle.fit import TABLE1
from oracle.pic import OracleSim
from oracle.steady import SteadyState

# lattice offsets of each component (E1..B3), per dimension, in cells
STAG3 = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]
NAMES = ("E1", "E2", "E3", "B1", "B2", "B3")


# ---- gather: quadratic fields reproduced per staggered component ----------------

@pytest.mark.parametrize("ndim", [2, 3])
def test_gather_reproduces_quadratic_field_per_component(ndim):
    n = (24, 20, 16)[:ndim]
    dx = (0.3, 0.5, 0.7)[:ndim]
    o = OracleSim(n, dx, 0.05)
    rng = np.random.default_rng(5)
    # positions well inside the grid (the stencil reaches two nodes each way)
    x = np.stack([rng.uniform(4.0, n[d] - 5.0, 64) for d in range(ndim)], axis=1)
    for c, name in enumerate(NAMES):
        st = STAG3[c][:ndim]
        for d in range(ndim):
            a, b, q = 0.7, -1.3 + 0.2 * c, 0.45 + 0.1 * d
            # the component's own coordinate along d at each lattice point
            idx = np.indices(tuple(reversed(n)))[ndim - 1 - d].astype(np.float64)
            X = idx + st[d]
            f = a + b * X + q * X * X
            # plus a separable bilinear term in two other coordinates
            if ndim >= 2:
                e = (d + 1) % ndim
                Y = np.indices(tuple(reversed(n)))[ndim - 1 - e].astype(np.float64) + st[e]
                f = f + 0.3 * X * Y
            fields = {nm: np.zeros(tuple(reversed(n))) for nm in NAMES}
            fields[name] = f
            for nm, arr in fields.items():
                o.set_field(nm, arr)
            got = o.gather_at(x)[:, c]
            xd = x[:, d]
            exact = a + b * xd + q * (xd * xd + 0.25)
            if ndim >= 2:
                exact = exact + 0.3 * xd * x[:, (d + 1) % ndim]
            assert np.abs(got - exact).max() < 1e-12 * np.abs(exact).max(), (name, d)
            # the other components read zero
            others = np.delete(o.gather_at(x), c, axis=1)
            assert np.abs(others).max() == 0.0


# ---- the lattice steady state of Sec. 2.1 is carried exactly ----------------------

STEADY_CASES = [
    # (solver, dx, [(x1, x2, Q, v)], (s, P), steps)
    ("yee", (1.0, 1.0), [(20.0, 16.0, 1.0, 1.0)], (1, 4), 40),
    ("custom", (1.0, 1.0), [(20.0, 16.0, 1.0, 1.0)], (1, 4), 40),
    # beta < 1, r != 1, two charges moving opposite ways, off-node starts
    ("yee", (1.0, 1.5), [(20.25, 8.0, 1.0, 0.75), (40.0, 20.5, -0.5, -0.5)], (3, 16), 48),
    ("custom", (1.0, 1.5), [(20.25, 8.0, 1.0, 0.75), (40.0, 20.5, -0.5, -0.5)], (3, 16), 48),
]


@pytest.mark.parametrize("solver,dx,parts,frac,steps", STEADY_CASES)
def test_pic_step_carries_the_lattice_steady_state(solver, dx, parts, frac, steps):
    n = (64, 32)
    dt = 0.25
    C = (1.0,) if solver == "yee" else tuple(TABLE1)
    ss = SteadyState(n, dx, dt, parts, frac, CE=C)
    assert ss.min_denominator() > 1e-12  # no exact resonance on this grid
    o = OracleSim(n, dx, dt, C=C)
    E1, E2, B3 = ss.fields(0)
    o.set_field("E1", E1)
    o.set_field("E2", E2)
    o.set_field("B3", B3)
    for (x1, x2, Q, v) in parts:
        # u large enough that u / gamma rounds to v exactly for |v| = 1
        u1 = math.copysign(1e8, v) if abs(v) == 1.0 else v / math.sqrt(1.0 - v * v)
        o.add_particles(np.array([[x1, x2]]), np.array([[u1, 0.0, 0.0]]), Q, 0.0)
    for k in (1, 2, 3, 5, steps):
        o.step(k - o.steps_done)
        ref = ss.fields(k)
        for nm, r in zip(("E1", "E2", "B3"), ref):
            got = o.field(nm)
            assert np.abs(got - r).max() < 1e-12 * np.abs(r).max(), (nm, k)
        for nm in ("E3", "B1", "B2"):
            assert np.abs(o.field(nm)).max() == 0.0


# ---- Yee self-force against the k-space F1 (Eq. 19) -------------------------------

def _window_self_force(n2, steps, C=(1.0,), filt=None):
    """A beta -> 1 unit charge on a node in a 64-cell window moving at c
    (kappa = 4, r = 1, dx = 1), ballistic; E1 line-out and F1 = Q E1(x_p)."""
    o = OracleSim((64, n2), (1.0, 1.0), 0.25, C=C, window=True, vwin=1.0)
    if filt is not None:
        o.set_filter(*filt)
    o.add_particles(np.array([[32.0, n2 / 2]]), np.array([[1e8, 0.0, 0.0]]), 1.0, 0.0)
    o.step(steps)
    x, _, alive = o.particles()
    assert alive[0]
    ip = int(round(x[0, 0])) - o.window_start
    assert abs(x[0, 0] - o.window_start - ip) < 1e-12  # on a node
    F1 = o.gather_at(x[:1])[0, 0]
    line = o.field("E1")[n2 // 2, ip - 3:ip + 2]  # E1 points i1' = -3..1
    return F1, line


@pytest.mark.slow
def test_yee_self_force_matches_kspace_integral():
    # Sec. 2.2: Yee, kappa = 4, r = 1, quadratic shape in both directions.
    # The periodic transverse grid shifts the field near the charge by
    # O(1/n2) (the x2-uniform mode of the charge and its start-up image);
    # runs at n2 = 32, 64, 128, each long enough to be steady near the
    # charge, are extrapolated to an unbounded grid (Richardson, error terms
    # 1/n2 and 1/n2^2) and compared with the k-space integral evaluated with
    # the same deposit (tpow 1 on axis) and the same gather (tpow 2, spline
    # weights at the E1 points).
    runs = {32: _window_self_force(32, 1200), 64: _window_self_force(64, 2400), 128: _window_self_force(128, 8000)}
    f = {k: v[0] for k, v in runs.items()}
    lines = {k: v[1] for k, v in runs.items()}
    F_inf = (8.0 * f[128] - 6.0 * f[64] + f[32]) / 3.0
    line_inf = (8.0 * lines[128] - 6.0 * lines[64] + lines[32]) / 3.0
    nus = (-3, -2, -1, 0, 1, 2, 3)
    F_th = kspace.KSpace("yee", 4.0, 1.0, order=2, beta=1.0, tpow=2, nus=nus).lattice_self_force()
    line_th = kspace.KSpace("yee", 4.0, 1.0, order=2, beta=1.0, tpow=1, nus=nus).e1(np.arange(-3, 2))
    assert abs(F_th + 0.0696) < 1e-4
    assert abs(F_inf - F_th) < 1e-3 * abs(F_th)
    assert np.abs(line_inf - line_th).max() < 4e-3 * np.abs(line_th).max()
    # the drag is decelerating and about a tenth of q^2/dx1 (Sec. 2.2: -0.10
    # for a linear transverse shape and the unaliased gather)
    assert -0.08 < f[128] < -0.06


@pytest.mark.slow
def test_fundamental_zone_cerenkov_yee_but_not_customized():
    # Table 2: Yee nu1 = 0 is Cerenkov-like (a steady drag: the field energy
    # grows at a constant rate as the wake is radiated); the customized
    # solver's fundamental zone carries no Cerenkov field, so once the
    # start-up radiation of a charge created in zero fields has been emitted
    # the field energy stops growing at the Yee rate.
    n, dx, dt = (512, 128), (1.0, 1.0), 0.25
    rates = {}
    for name, C in (("yee", (1.0,)), ("custom", tuple(TABLE1))):
        o = OracleSim(n, dx, dt, C=C)
        o.add_particles(np.array([[16.0, 64.0]]), np.array([[1e8, 0.0, 0.0]]), 1.0, 0.0)
        w = []
        for N in (200, 400, 800, 1200):
            o.step(N - o.steps_done)
            w.append(o.energy()[0])
        rates[name] = [(w[i + 1] - w[i]) / (dt * d) for i, d in enumerate((200, 400, 400))]
    yee, cus = rates["yee"], rates["custom"]
    assert abs(yee[-1] - yee[0]) < 0.1 * yee[0]            # steady radiation
    assert 0.05 < yee[-1] < 0.12                            # of order |F1| c
    assert cus[-1] < 0.25 * yee[-1]                         # no steady drag
    assert cus[-1] < 0.7 * cus[0]                           # and still falling


# ---- the 5-pass current filter ----------------------------------------------------

FIVE_PASS = (4, 5.0)


def test_current_filter_symbol():
    # four (1, 2, 1)/4 passes and the compensator (-5/4, 7/2, -5/4) along x1:
    # a Fourier mode of the current is multiplied by cos^8(k dx1/2) (1 + 5 sin^2(k dx1/2))
    n1 = 64
    o = OracleSim((n1, 4), (1.0, 1.0), 0.25)
    o.set_filter(*FIVE_PASS)
    i1 = np.arange(n1)
    for m in (1, 5, 16, 31):
        k = 2 * np.pi * m / n1
        f = np.cos(k * i1 + 0.3)[None, :] * np.ones((4, 1))
        for nm in ("J1", "J2", "J3"):
            o.set_field(nm, f)
        o.filter_j()
        sym = np.cos(k / 2) ** 8 * (1 + 5 * np.sin(k / 2) ** 2)
        for nm in ("J1", "J2", "J3"):
            assert np.abs(o.field(nm) - sym * f).max() < 1e-14


def test_gauss_law_with_the_filter_holds_for_the_filtered_density():
    rng = np.random.default_rng(5)
    n, dx = (64, 16), (1.0, 1.2)
    o = OracleSim(n, dx, 0.25, C=tuple(TABLE1))
    o.set_filter(*FIVE_PASS)
    X = np.stack([rng.uniform(0, n[0], 40), rng.uniform(0, n[1], 40)], axis=1)
    u = rng.normal(0, 2.0, (40, 3))
    u[:, 0] += 3.0
    o.add_particles(X, u, -0.3, -1.0)

    def filtered(rho):
        k = 2 * np.pi * np.fft.fftfreq(n[0])
        sym = np.cos(k / 2) ** 8 * (1 + 5 * np.sin(k / 2) ** 2)
        return np.real(np.fft.ifft(np.fft.fft(rho, axis=-1) * sym, axis=-1))

    r0 = o.div_e() - filtered(o.rho())
    o.step(12)
    r1 = o.div_e() - filtered(o.rho())
    assert np.abs(r1 - r0).max() < 1e-12 * np.abs(o.rho()).max()
    assert np.abs(o.field("E1")).max() > 0


@pytest.mark.slow
def test_filtered_yee_self_force_matches_kspace_integral():
    # as the unfiltered pin, with the current smoothed: the k-space F1 of the
    # same filter (whose paper-convention value reproduces the printed -0.031)
    f = {n2: _window_self_force(n2, st, filt=FIVE_PASS)[0] for n2, st in ((32, 1200), (64, 2400), (128, 8000))}
    F_inf = (8.0 * f[128] - 6.0 * f[64] + f[32]) / 3.0
    nus = tuple(range(-3, 4))
    F_th = kspace.KSpace("yee", 4.0, 1.0, order=2, beta=1.0, tpow=2, nus=nus, filt=FIVE_PASS).lattice_self_force()
    assert abs(F_inf - F_th) < 1e-3 * abs(F_th), (f, F_inf, F_th)
    # the filter cuts the Yee drag by two thirds (Sec. 2.2: -0.10 -> -0.031 in the paper's convention)
    f0 = _window_self_force(32, 1200)[0]
    assert abs(f[32]) < 0.6 * abs(f0)
