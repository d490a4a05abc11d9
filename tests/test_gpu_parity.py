"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
identical seeded inputs.  Bar: FP64 fields and particles within 1e-12
(relative to each component's maximum), FP32 fields within 1e-5."""
import math

import numpy as np
import pytest

from oracle import dispersion, fit
from paper_1910_13529_amd import inputs
from tests.gpu_common import CANCEL_FRACTION, beam_species, field_errors, log, make_pair, particle_errors

pytestmark = pytest.mark.gpu

TABLE1 = tuple(fit.TABLE1)


def test_single_particle_2d_fp64():
    # one macro-electron, gamma = 1000, on node (64, 64) of a periodic 256x128
    # grid, dx = 0.05, dt = 0.9 Courant, quadratic shape, Yee, 400 steps
    w = inputs.config_single_particle()
    cell, off, u = inputs.single_particle(w.extra["node"], w.extra["gamma"])
    g, o, ids = make_pair(2, w.n, w.dx, w.dt, (1.0,), False, [(-1.0, -1.0, cell, off, u, 1)])
    done = 0
    for stop in (1, 50, 400):
        log("single-particle fp64: step %d" % stop)
        g.step(stop - done)
        o.step(stop - done)
        done = stop
        errs = field_errors(g, o)
        assert max(errs.values()) < 1e-12, (stop, errs)
        dxp, dup = particle_errors(g, o, ids[0], 1)
        assert dxp < 1e-12 and dup < 1e-12, (stop, dxp, dup)
    g.sync()


def test_beam_2d_custom_periodic_fp64():
    n, dx, dt = (128, 32), (1.0, 1.0), 0.25
    sp = beam_species(7, 300, n, dx, 20.0, Q=-0.05, sigma_cells=(6.0, 2.0), divergence=0.05, espread=0.05)
    g, o, ids = make_pair(2, n, dx, dt, TABLE1, False, [sp])
    assert g.correction_halfwidth > 30
    g.step(60)
    o.step(60)
    errs = field_errors(g, o)
    log("beam 2d custom fp64: %s" % errs)
    assert max(errs.values()) < 1e-12, errs
    dxp, dup = particle_errors(g, o, ids[0], 300)
    assert dxp < 1e-12 and dup < 1e-12
    g.sync()


@pytest.mark.parametrize("solver", ["yee", "custom"])
@pytest.mark.parametrize("precision,tol,ptol", [("fp64", 1e-12, 1e-12), ("fp32", 1e-5, 2e-5)])
def test_beam_3d_window(solver, precision, tol, ptol):
    n, dx, dt = (72, 16, 16), (0.02, 0.05, 0.05), 0.005
    C = (1.0,) if solver == "yee" else TABLE1
    sp = beam_species(3, 2000, n, dx, 1e4, Q=-1e-3, sigma_cells=(5.0, 1.0, 1.0), center_frac=0.6)
    g, o, ids = make_pair(3, n, dx, dt, C, True, [sp], precision=precision)
    g.step(41)
    o.step(41)
    assert g.get_step() == (41, 10)
    assert o.window_start == 10
    errs = field_errors(g, o)
    log("beam 3d window %s %s: %s" % (solver, precision, errs))
    assert max(errs.values()) < tol, errs
    dxp, dup = particle_errors(g, o, ids[0], 2000)
    assert dxp < ptol and dup < ptol, (dxp, dup)
    g.sync()


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("solver", ["yee", "custom"])
def test_vacuum_dispersion_gpu(ndim, solver):
    # an exact discrete eigenmode advances as cos(omega n dt) with omega from
    # sin^2(omega dt/2) = (dt/2)^2 sum [k]^2 (Eq. 4)
    from paper_1910_13529_amd.relpic import Sim
    C = (1.0,) if solver == "yee" else TABLE1
    if ndim == 2:
        n, dx, dt, m = (48, 16), (1.0, 0.8), 0.25, (5, 3)
    else:
        n, dx, dt, m = (40, 4, 12), (1.0, 1.0, 0.9), 0.25, (4, 0, 2)
    grid = dict(ndim=ndim, n=n + (1,) * (3 - ndim), dx=dx + (1.0,) * (3 - ndim), dt=dt)
    g = Sim(grid, C=list(C) if len(C) > 1 else None, precision="fp64")
    k = [2 * math.pi * m[d] / (n[d] * dx[d]) for d in range(ndim)]
    idx = np.meshgrid(*[np.arange(n[d]) for d in reversed(range(ndim))], indexing="ij")
    pos = [idx[ndim - 1 - d] * dx[d] for d in range(ndim)]
    if ndim == 2:
        basis = np.cos(k[0] * pos[0] + k[1] * pos[1])
        comp, kk, dd = "E3", (k[0], k[1]), (dx[0], dx[1])
    else:
        basis = np.cos(k[0] * pos[0] + k[2] * pos[2])
        comp, kk, dd = "E2", (k[0], k[2]), (dx[0], dx[2])
    g.set_field(comp, basis)
    w = dispersion.omega(kk, dd, dt, C1=C)
    worst = 0.0
    for it in range(1, 121):
        g.step(1)
        if it % 20 == 0:
            amp = (g.field(comp) * basis).sum() / (basis * basis).sum()
            worst = max(worst, abs(amp - math.cos(w * it * dt)))
    assert worst < 1e-12


def test_gauss_and_energy_diagnostics_fp64():
    n, dx, dt = (96, 24), (1.0, 1.0), 0.25
    sp = beam_species(9, 400, n, dx, 5.0, Q=-0.05, sigma_cells=(5.0, 2.0), divergence=0.1, espread=0.1)
    g, o, ids = make_pair(2, n, dx, dt, TABLE1, False, [sp])
    g.set_background_rho(-o.rho())  # immobile neutralizing background = minus the t=0 density
    d0 = g.diagnostics()
    assert d0["rho_max"] > 0 and d0["gauss_max"] < 1e-13 * d0["rho_max"]
    assert abs(d0["charge"] - 400 * -0.05) < 1e-12
    g.step(30)
    o.step(30)
    d = g.diagnostics()
    assert d["gauss_max"] < 1e-12 * d["rho_max"]
    wf, wk = o.energy()
    assert abs(d["w_field"] - wf) < 1e-11 * wf
    assert abs(d["w_kin"] - wk) < 1e-12 * abs(wk)
    assert d["n_alive"] == 400 and d["error_word"] == 0


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("layout", ["bunch_sorted", "bunch_unsorted", "scattered"])
def test_rho_diagnostic_layouts_fp64(ndim, layout):
    # the diagnostic's charge density node by node against the oracle's: with
    # zero fields and the background set to minus the oracle's rho, the Gauss
    # residual is rho_gpu - rho_oracle.  A sorted or unsorted bunch sums in the
    # workgroups' LDS tiles; particles scattered over the whole grid (chunk
    # boxes larger than the tile) add to rho directly.
    if ndim == 3:
        n, dx, window = (72, 16, 16), (0.02, 0.05, 0.05), layout != "scattered"
    else:
        n, dx, window = (256, 64), (1.0, 1.0), False
    if layout == "scattered":
        cell, off, u = inputs.uniform_particles(13, 30000, n, 1e-3, ndim=ndim)
        sp = (-1e-3, -1.0, cell, off, u, len(cell))
    else:
        sp = beam_species(11, 30000, n, dx, 100.0, Q=-1e-3, sigma_cells=(5.0, 2.0, 2.0)[:ndim], center_frac=0.5)
    npart = len(sp[2])
    # Yee operator: the window's excluded edge (2M + 2 cells) is then 4 cells
    g, o, ids = make_pair(ndim, n, dx, 0.005, (1.0,), window, [sp])
    if layout == "bunch_sorted":
        g.sort_particles()
    g.set_background_rho(-o.rho())
    log("rho diagnostic %dD %s" % (ndim, layout))
    d = g.diagnostics()
    assert d["rho_max"] > 0 and d["gauss_max"] < 1e-13 * d["rho_max"], d
    assert abs(d["charge"] - npart * -1e-3) < 1e-12 * npart * 1e-3
    g.sync()


def _beam_sim(n, dx, dt, C, window, sp, precision):
    from paper_1910_13529_amd.relpic import Sim
    grid = dict(ndim=3, n=tuple(n), dx=tuple(dx), dt=dt, window=window, window_speed=1.0)
    g = Sim(grid, C=list(C) if len(C) > 1 else None, precision=precision)
    Q, qm, cell, off, u, cap = sp
    sid = g.add_species(qm, Q, cap)
    g.load_particles(sid, cell, off, u)
    return g, sid


@pytest.mark.parametrize("solver", ["yee", "custom"])
@pytest.mark.parametrize("window", [False, True])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_fused_field_update_matches_separate(solver, window, precision, tol):
    # the fused E and B update (one pass per step) against the separate
    # updates on the same run: n3 = 44 is five full columns of 8 planes and a
    # partial one, the window shifts every 2.5 steps (the fused result is
    # carried to the shifted window), and calls of 7, 1, 1 and 12 steps end
    # with the fused epilogue
    n, dx, dt = (64, 12, 44), (0.5, 1.0, 1.0), 0.2
    C = (1.0,) if solver == "yee" else TABLE1
    sp = beam_species(5, 3000, n, dx, 50.0, Q=-0.02, sigma_cells=(4.0, 1.5, 1.5), center_frac=0.5,
                      divergence=0.02, espread=0.02)
    fields = {}
    for fused in (True, False):
        g, sid = _beam_sim(n, dx, dt, C, window, sp, precision)
        assert g.set_fused_fields(fused) == fused
        for k in (7, 1, 1, 12):
            g.step(k)
        fields[fused] = {nm: g.field(nm) for nm in ("E1", "E2", "E3", "B1", "B2", "B3")}
        fields[fused]["x"] = g.particles(sid, 3000)
        g.sync()
    log("fused vs separate %s window=%s %s" % (solver, window, precision))
    for grp in ("E", "B"):
        gmax = max(float(np.abs(fields[False][grp + c]).max()) for c in "123")
        for c in "123":
            own = float(np.abs(fields[False][grp + c]).max())
            assert own > 0
            scale = own if own >= CANCEL_FRACTION * gmax else gmax  # cancelling component: its terms' scale
            d = float(np.abs(fields[True][grp + c] - fields[False][grp + c]).max())
            log("  %s%s: %.3g of %s maximum" % (grp, c, d / scale, "its" if scale == own else "the field's"))
            assert d <= tol * scale, (grp + c, d, scale)
    (ca, oa, ua, aa), (cb, ob, ub, ab) = fields[True]["x"], fields[False]["x"]
    assert (aa == ab).all()
    assert np.abs((ca + oa) - (cb + ob))[aa].max() < 10 * tol


def test_fused_field_update_availability():
    from paper_1910_13529_amd.relpic import RelpicError, Sim
    g3 = Sim(dict(ndim=3, n=(64, 8, 8), dx=(1.0, 1.0, 1.0), dt=0.3), precision="fp32")
    assert g3.set_fused_fields(True)
    assert not g3.set_fused_fields(False)
    g2 = Sim(dict(ndim=2, n=(64, 8, 1), dx=(1.0, 1.0, 1.0), dt=0.3), precision="fp32")
    with pytest.raises(RelpicError):
        g2.set_fused_fields(True)
    assert not g2.set_fused_fields(False)
    # odd x2 extent (the row block is two rows)
    g3b = Sim(dict(ndim=3, n=(64, 7, 8), dx=(1.0, 1.0, 1.0), dt=0.3), precision="fp32")
    with pytest.raises(RelpicError):
        g3b.set_fused_fields(True)


@pytest.mark.parametrize("precision,tol,xtol,utol,steps,sort_every,n", [
    ("fp64", 1e-12, 1e-12, 1e-13, 13, 0, (40, 8, 8)), ("fp64", 1e-12, 1e-12, 1e-13, 30, 5, (40, 8, 8)),
    ("fp32", 1e-5, 2e-5, 2e-5, 30, 5, (40, 8, 8)), ("fp64", 1e-12, 1e-12, 1e-13, 13, 0, (40, 12, 10)),
    ("fp32", 1e-5, 2e-5, 2e-5, 30, 5, (40, 20, 13))])
def test_plasma_injection_window(precision, tol, xtol, utol, steps, sort_every, n):
    # cold plasma ahead of a beam in the moving window: the window injects a
    # slab of 2x2x2 particles per cell at each shift, momenta from the shared
    # counter-based generator, its cells stored in 8x8 transverse blocks
    # (narrower at the ends on the ragged grids).  With re-sorts every few
    # steps the plasma is sorted by tiles of storage cells after the window
    # has moved (ring buffer offset), and in FP32 deposits with the wide
    # rounds.
    dx, dt = (0.02, 0.05, 0.05), 0.005
    cellp, offp, up = inputs.plasma_lattice(4, (2, 0, 0), (n[0] - 2, n[1], n[2]), (2, 2, 2), 1e-4)
    keep = cellp[:, 0] <= n[0] - 3
    cellp, offp, up = cellp[keep], offp[keep], up[keep]
    Qp = -(0.02 * 0.05 * 0.05) / 8.0
    nplasma = len(cellp)
    inj_per_shift = 8 * n[1] * n[2]
    shifts = steps // 4
    cap = nplasma + (shifts + 1) * inj_per_shift
    beam = beam_species(5, 300, n, dx, 1e4, Q=-1e-4, sigma_cells=(3.0, 1.0, 1.0), center_frac=0.5)
    g, o, ids = make_pair(3, n, dx, dt, TABLE1, True, [beam, (Qp, -1.0, cellp, offp, up, cap)], precision=precision)
    g.set_injection(ids[1], (2, 2, 2), 1e-4, 1234)
    o.set_injection((2, 2, 2), Qp, -1.0, 1e-4, 1234)
    if sort_every:
        g.set_sort_interval(sort_every)
    g.step(steps)
    o.step(steps)
    errs = field_errors(g, o)
    log("plasma injection %s, %d steps, sort every %d: %s" % (precision, steps, sort_every, errs))
    assert max(errs.values()) < tol, errs
    # oracle stores both species in one list: beam first, then plasma
    # (particle ids: load order, then injection order); a re-sort drops the
    # particles that left the window, which the oracle keeps as dead slots
    xo, uo, ao = o.particles()
    xo, uo, ao = xo[300:], uo[300:], ao[300:]
    assert len(ao) == nplasma + shifts * inj_per_shift
    cell, off, u, alive = g.particles(ids[1], cap)
    gid = g.last_ids[alive]
    assert np.array_equal(gid, np.flatnonzero(ao))
    xg = cell[alive].astype(np.float64) + off[alive]
    dxm = float(np.abs(xg - xo[gid]).max())
    # momenta against the largest plasma momentum (the beam's field kicks the
    # plasma electrons from u_th = 1e-4 to a few 1e-2)
    umax = float(np.abs(uo[gid]).max())
    dum = float(np.abs(u[alive] - uo[gid]).max()) / umax
    log("  plasma particles: max |dx| %.3g cells, max |du|/max |u| %.3g (max |u| %.3g)" % (dxm, dum, umax))
    assert dxm < xtol and dum < utol


@pytest.mark.parametrize("ndim", [3, 2])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_dense_bunch(ndim, precision, tol):
    """A bunch packed into one transverse cell and a few x1 cells (thousands
    of particles per cell, as in the core of a dense beam): whole wavefronts
    share one cell and deposit through the wavefront reduce-scatter."""
    n = (64, 12, 12)[:ndim]
    dx = (0.02, 0.05, 0.05)[:ndim]
    dt = 0.005
    center = [0.5 * n[0]] + [n[d] // 2 for d in range(1, ndim)]
    cell, off, u = inputs.gaussian_bunch(21, 12000, center, (0.6,) + (0.08,) * (ndim - 1), 1e4, 0.01, 1e-3,
                                         ndim=ndim, clip_sigmas=4.0)
    sp = (-1e-4, -1.0, cell, off, u, len(cell))
    g, o, ids = make_pair(ndim, n, dx, dt, TABLE1, False, [sp], precision=precision)
    g.step(30)
    o.step(30)
    errs = field_errors(g, o)
    log("dense bunch %dD %s: %s" % (ndim, precision, errs))
    assert max(errs.values()) < tol, errs
    dxp, dup = particle_errors(g, o, ids[0], len(cell))
    assert dxp < (1e-12 if precision == "fp64" else 1e-4) and dup < tol * 2
    g.sync()


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("precision,tol,ptol", [("fp64", 1e-12, 1e-12), ("fp32", 1e-5, 2e-5)])
def test_sort_key_order_by_density(ndim, precision, tol, ptol):
    # the sort groups a sparse species (about two particles per cell over the
    # whole grid) by w x 4 (x 4) tiles of cells, x1 fastest inside a tile (w =
    # 8 in FP32, 4 in FP64), and a dense bunch (hundreds per occupied cell) by
    # rows; either order keeps every particle once and each cell's particles
    # together, and the steps that follow (wide deposit rounds for the sparse
    # species in FP32) match the oracle.  The grid is ragged against the
    # tiles in every axis.
    n = (76, 22, 14)[:ndim]
    dx = (0.5, 1.0, 1.0)[:ndim]
    ncell = int(np.prod(n))
    cs, os_, us = inputs.uniform_particles(21, 2 * ncell, n, 1e-2, ndim=ndim)
    sparse = (-1e-4, -1.0, cs, os_, us, len(cs))
    dense = beam_species(22, 20000, n, dx, 20.0, Q=-1e-4, sigma_cells=(1.5, 0.5, 0.5), center_frac=0.5)
    g, o, ids = make_pair(ndim, n, dx, 0.2, (1.0,), False, [sparse, dense], precision=precision)
    g.sort_particles()
    w1 = 8 if precision == "fp32" else 4

    def row_key(c):
        k = c[:, ndim - 1].astype(np.int64)
        for d in range(ndim - 2, -1, -1):
            k = k * n[d] + c[:, d]
        return k

    def tile_key(c):
        nt = [(n[0] + w1 - 1) // w1] + [(n[d] + 3) // 4 for d in range(1, ndim)]
        tile = c[:, ndim - 1].astype(np.int64) // 4
        local = c[:, ndim - 1].astype(np.int64) % 4
        for d in range(ndim - 2, -1, -1):
            w = w1 if d == 0 else 4
            tile = tile * nt[d] + c[:, d] // w
            local = local * w + c[:, d] % w
        return tile * (w1 * 4 ** (ndim - 1)) + local

    for sid, (_, _, cell0, _, _, cap), tiled in ((ids[0], sparse, True), (ids[1], dense, False)):
        cell, off, u, alive = g.particles(sid, cap, order_by_id=False)
        assert alive.all() and len(cell) == len(cell0)
        assert sorted(g.last_ids.tolist()) == list(range(len(cell0)))
        key = tile_key(cell) if tiled else row_key(cell)
        assert (np.diff(key) >= 0).all()
        if tiled:
            assert (np.diff(row_key(cell)) < 0).any()  # not row order
        log("sort order %dD %s: %d particles, %d cells" % (ndim, "tiles" if tiled else "rows", len(cell),
                                                          len(np.unique(key))))
    for _ in range(3):
        g.step(1)
        o.step(1)
    errs = field_errors(g, o)
    log("sort order %dD %s: fields %s" % (ndim, precision, errs))
    assert max(errs.values()) < tol, errs
    xo, uo, ao = o.particles()
    assert ao.all()
    nn = np.asarray(n, dtype=np.float64)[None, :]
    start = 0
    for sid, sp in zip(ids, (sparse, dense)):
        cell, off, u, alive = g.particles(sid, sp[5])
        sl = slice(start, start + sp[5])
        start += sp[5]
        d = (cell + off) - xo[sl]
        d = (d + nn / 2) % nn - nn / 2  # periodic wrap
        du = np.linalg.norm(u - uo[sl], axis=1) / np.maximum(np.linalg.norm(uo[sl], axis=1), 1e-300)
        log("  species %d: max |dx| %.3g cells, max |du|/|u| %.3g" % (sid, float(np.abs(d).max()), float(du.max())))
        assert alive.all() and float(np.abs(d).max()) < ptol and float(du.max()) < ptol
    g.close()
    o.close()


@pytest.mark.parametrize("precision,limit", [("fp32", 1 << 30), ("fp64", 1 << 29)])
def test_species_capacity_limit(precision, limit):
    # the push addresses each particle array with 32-bit byte offsets, so a
    # species holds at most 2^32 bytes per array; the check happens before
    # any allocation (the limit itself is not allocated here)
    from paper_1910_13529_amd.relpic import RelpicError, Sim
    g = Sim(dict(ndim=3, n=(16, 8, 8), dx=(1.0, 1.0, 1.0), dt=0.3), precision=precision)
    with pytest.raises(RelpicError):
        g.add_species(-1.0, -1e-3, limit + 1)
    g.add_species(-1.0, -1e-3, 1024)
    g.close()

@pytest.mark.parametrize("sort_every", [25, 2])
def test_grouped_deposit_irregular_runs(sort_every):
    # FP32 tile-sorted species whose cells hold irregular particle counts
    # (most 8, some Poisson around 8, some 1-3, some 12-20 (runs cut into
    # pieces of 8), and a sparse slab of 1-2 per cell at small x3), so push
    # chunks (1024 particles, K = 4) are walked by cell groups over 4-5
    # iterations, or in array order where their runs make more than 160
    # groups; thermal momenta move a share of the particles across x1 and
    # transverse cell faces each step (their lanes leave the group sums for
    # the rounds or the direct path), and the steps between re-sorts split
    # runs further.  Fields and particles against the oracle.
    n, dx, dt = (64, 32, 32), (0.5, 1.0, 1.0), 0.2
    rng = np.random.default_rng(31)
    counts = np.full(n, 8, dtype=np.int64)
    r = rng.uniform(size=n)
    pois = rng.poisson(8.0, size=n)
    few = rng.integers(1, 4, size=n)
    many = rng.integers(12, 21, size=n)
    counts = np.where(r < 0.3, np.maximum(pois, 1), counts)
    counts = np.where((r >= 0.3) & (r < 0.4), few, counts)
    counts = np.where((r >= 0.4) & (r < 0.5), many, counts)
    counts[:, :, :6] = rng.integers(1, 3, size=(n[0], n[1], 6))
    cell, off, u = inputs.cells_with_counts(32, counts, 0.3)
    sp = (-1e-4, -1.0, cell, off, u, len(cell))
    log("grouped deposit: %d particles in %d cells, sort every %d" % (len(cell), counts.size, sort_every))
    g, o, ids = make_pair(3, n, dx, dt, TABLE1, False, [sp], precision="fp32")
    g.set_sort_interval(sort_every)
    steps = 5
    g.step(steps)
    o.step(steps)
    errs = field_errors(g, o)
    log("grouped deposit, sort every %d: fields %s" % (sort_every, errs))
    assert max(errs.values()) < 1e-5, errs
    xo, uo, ao = o.particles()
    assert ao.all()
    c, of, ug, alive = g.particles(ids[0], len(cell))
    assert alive.all()
    nn = np.asarray(n, dtype=np.float64)[None, :]
    d = (c + of) - xo
    d = (d + nn / 2) % nn - nn / 2
    du = np.linalg.norm(ug - uo, axis=1) / np.maximum(np.linalg.norm(uo, axis=1), 1e-300)
    log("  particles: max |dx| %.3g cells, max |du|/|u| %.3g" % (float(np.abs(d).max()), float(du.max())))
    assert float(np.abs(d).max()) < 2e-5 and float(du.max()) < 2e-5
    g.close()
    o.close()
