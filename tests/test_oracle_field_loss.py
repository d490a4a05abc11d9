"""Pins of the oracle's field loss (oracle/field_loss.py) against brute-force
counts and closed forms, and of its total loss's quadratic dependence on the
bunch charge."""
import numpy as np

from oracle import field_loss
from paper_1910_13529_amd import workloads

BOX = dict(x1=1.0, x2=0.6, v1=1.0, half1=0.3, half2=0.15)


def brute(E1, E2, B3, n, box, dx, dt):
    n2, n1 = E1.shape
    c1 = box["x1"] + box["v1"] * n * dt
    tot = 0.0
    for i2 in range(n2):
        for i1 in range(n1):
            x1, x2 = (i1 + 0.5) * dx[0], i2 * dx[1]
            if abs(x1 - c1) > box["half1"] or abs(x2 - box["x2"]) > box["half2"]:
                tot += E1[i2, i1] ** 2
            x1, x2 = i1 * dx[0], (i2 + 0.5) * dx[1]
            if abs(x1 - c1) > box["half1"] or abs(x2 - box["x2"]) > box["half2"]:
                b3c = 0.5 * (B3[i2, i1 - 1] + B3[i2, i1])  # i1 - 1 = -1 wraps to the last column
                tot += (E2[i2, i1] - b3c) ** 2
    return tot * dx[0] * dx[1] * dt


def test_step_loss_matches_brute_force_sum():
    rng = np.random.default_rng(5)
    shape = (24, 40)
    E1, E2, B3 = (rng.standard_normal(shape) for _ in range(3))
    dx, dt = (0.05, 0.05), 0.0125
    for n in (0, 3, 17):
        a = field_loss.step_loss(E1, E2, B3, n, BOX, dx, dt)
        b = brute(E1, E2, B3, n, BOX, dx, dt)
        assert abs(a - b) < 1e-12 * abs(b)


def test_step_loss_counts_points_outside_the_box():
    """E1 = 1, E2 = B3 = 0: the loss is w times the number of E1 points outside
    the box; the box of half-widths 0.3 x 0.16 around (1.0, 0.6) holds 12 x 7
    E1 points (x1 = 0.725 .. 1.275, x2 = 0.45 .. 0.75)."""
    shape = (24, 40)
    dx, dt = (0.05, 0.05), 0.01
    E1 = np.ones(shape)
    Z = np.zeros(shape)
    box = dict(BOX, half2=0.16)
    L = field_loss.step_loss(E1, Z, Z, 0, box, dx, dt)
    inside = 12 * 7
    assert abs(L - dx[0] * dx[1] * dt * (shape[0] * shape[1] - inside)) < 1e-15


def test_beta_one_field_pair_has_zero_loss():
    """E2 equal to B3 moved onto E2's point (E2 - B3c = 0) contributes nothing;
    a B3 ramp a * (i1 + 1/2) averages to a * i1 except across the periodic seam."""
    shape = (16, 32)
    dx, dt = (0.05, 0.05), 0.01
    a = 0.37
    i1 = np.arange(shape[1])[None, :] * np.ones(shape)
    B3 = a * (i1 + 0.5)
    E2 = a * i1
    Z = np.zeros(shape)
    far = dict(x1=100.0, x2=100.0, v1=0.0, half1=0.01, half2=0.01)  # nothing excluded
    L = field_loss.step_loss(Z, E2, B3, 0, far, dx, dt)
    # only column i1 = 0 differs: B3c(0) = (a (n1 - 1/2) + a/2) / 2 = a n1 / 2
    r0 = a * shape[1] / 2.0
    assert abs(L - dx[0] * dx[1] * dt * shape[0] * r0 * r0) < 1e-12 * L


def test_total_loss_is_quadratic_in_the_charge():
    w = workloads.adjoint_workload(n=(64, 32), npart=256, nsteps=12, M=1)
    L1 = field_loss.total_loss(w, [1.0])
    w2 = dict(w)
    w2["Q"] = 2.0 * w["Q"]
    L2 = field_loss.total_loss(w2, [1.0])
    assert L1 > 0
    assert abs(L2 / L1 - 4.0) < 1e-10
