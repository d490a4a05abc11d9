"""Element-by-element parity against the FP64 oracle at the configurations
themselves (not only on small grids):

* the 3D beam at 512 x 256 x 256 with 2^22 particles, FP32, customized
  solver (Table 1), fused field update -- the launch configuration the
  benchmark times -- for 5 steps including a window shift: every field
  component within 1e-5 and every particle against the oracle's;
* three of the 256 batched runs at their real sizes (up to 1024 x 256,
  4096 particles each), advanced inside the full batch, against the oracle;
* a beam in a plasma at 8 particles per cell over the whole grid (the
  plasma workload's make-up at a reduced grid): tile-sorted plasma with the
  wide deposit rounds in FP32, current over the whole grid (so the J1
  correction runs on every x1 line), injection at every window shift, in
  FP32 and FP64.

The oracle runs its field loops and its gather + push on every host core
(OpenMP); its deposit stays serial."""
import numpy as np
import pytest

from oracle import fit
from oracle.pic import OracleSim
from paper_1910_13529_amd import inputs, workloads
from tests.gpu_common import field_errors, log

pytestmark = pytest.mark.gpu

TABLE1 = tuple(fit.TABLE1)
TILE_CELLS_FP32 = 49152 // (9 * 4)  # cells of the push's LDS tile (E, B and J)


def _hbm_fallback_chunks(cell, n, K):
    """Push chunks (256 K consecutive particles in cell order) whose box of
    old cells +- 2 does not fit the LDS tile: those gather from and deposit to
    HBM directly."""
    key = cell[:, 0] + n[0] * (cell[:, 1] + n[1] * cell[:, 2])
    c = cell[np.argsort(key, kind="stable")]
    m = 256 * K
    count = 0
    for s in range(0, len(c), m):
        blk = c[s:s + m]
        ext = (blk.max(axis=0) - blk.min(axis=0)) + 5
        if int(np.prod(ext)) > TILE_CELLS_FP32:
            count += 1
    return count


def test_fullsize_beam3d_elementwise_fp32():
    from paper_1910_13529_amd.relpic import Sim
    w = inputs.config_beam3d(n=(512, 256, 256))
    cell, off, u = inputs.beam_inputs(w, seed=2)
    Q = inputs.beam_charge(w)
    n = len(cell)
    log("full-size beam: %d particles, %d HBM-fallback chunks at K = 4" % (n, _hbm_fallback_chunks(cell, w.n, 4)))
    grid = dict(ndim=3, n=w.n, dx=w.dx, dt=w.dt, window=True, window_speed=1.0)
    g = Sim(grid, C=list(TABLE1), precision="fp32")
    assert g.set_fused_fields(True)
    sid = g.add_species(-1.0, Q, n)
    g.load_particles(sid, cell, off, u)
    o = OracleSim(w.n, w.dx, w.dt, C=TABLE1, window=True)
    o.add_particles(cell.astype(np.float64) + off, u, Q, -1.0)
    steps = 5  # the window shifts after step 4
    g.step(steps)
    log("full-size beam: oracle, %d steps" % steps)
    for k in range(steps):
        o.step(1)
        log("  oracle step %d done" % (k + 1))
    assert o.window_start == 1 and g.get_step() == (steps, 1)
    errs = field_errors(g, o)
    log("full-size beam fields: %s" % errs)
    assert max(errs.values()) < 1e-5, errs
    c, of, uu, alive = g.particles(sid, n)
    xo, uo, ao = o.particles()
    assert alive.all() and ao.all()
    dxm = float(np.abs((c + of) - xo).max())
    dum = float((np.linalg.norm(uu - uo, axis=1) / np.linalg.norm(uo, axis=1)).max())
    log("full-size beam particles: max |dx| %.3g cells, max |du|/|u| %.3g" % (dxm, dum))
    assert dxm < 2e-5 and dum < 2e-6  # FP32 state against the FP64 oracle
    g.close()
    o.close()


def test_batch_runs_at_real_size_vs_oracle_fp32():
    runs = workloads.batch_workload(256)
    big = max(range(256), key=lambda k: runs[k]["grid"]["n"][0] * runs[k]["grid"]["n"][1])
    cus = next(k for k in range(256) if runs[k]["C"] is not None and k != big)
    yee = next(k for k in range(256) if runs[k]["C"] is None and k != big)
    from paper_1910_13529_amd.relpic import Batch
    b = Batch([r["grid"] for r in runs], [r["C"] for r in runs], precision="fp32")
    for br, r in zip(b.runs, runs):
        sid = br.add_species(-1.0, r["Q"], len(r["cell"]))
        br.load_particles(sid, r["cell"], r["offset"], r["u"])
    steps = 20
    b.step(steps)
    b.sync()
    for k in (big, cus, yee):
        r = runs[k]
        gr = r["grid"]
        nn = (gr["n"][0], gr["n"][1])
        o = OracleSim(nn, gr["dx"][:2], gr["dt"], C=tuple(r["C"]) if r["C"] is not None else (1.0,))
        o.add_particles(r["cell"].astype(np.float64) + r["offset"], r["u"], r["Q"], -1.0)
        o.step(steps)
        errs = field_errors(b.runs[k], o)
        log("batched run %d (%dx%d, %s): %s" % (k, nn[0], nn[1], "custom" if r["C"] is not None else "Yee", errs))
        assert max(errs.values()) < 1e-5, (k, errs)
        o.close()
    b.close()


@pytest.mark.parametrize("precision,tol,ptol", [("fp32", 1e-5, 2e-5), ("fp64", 1e-12, 1e-12)])
def test_plasma_whole_grid_vs_oracle(precision, tol, ptol):
    from paper_1910_13529_amd.relpic import Sim
    n, dx, dt = (96, 32, 32), (0.02, 0.05, 0.05), 0.005
    dV = dx[0] * dx[1] * dx[2]
    Qp = -dV / 8.0
    cellp, offp, up = inputs.plasma_lattice(8, (2, 0, 0), (n[0] - 2, n[1], n[2]), (2, 2, 2), 1e-4)
    keep = cellp[:, 0] <= n[0] - 3
    cellp, offp, up = cellp[keep], offp[keep], up[keep]
    beam_c, beam_o, beam_u = inputs.gaussian_bunch(9, 20000, (0.6 * n[0], n[1] / 2, n[2] / 2), (4.0, 1.0, 1.0), 1e4,
                                                   0.01, 1e-3, ndim=3, clip_sigmas=3.0)
    Qb = -1e-3
    steps = 10
    inj = 8 * n[1] * n[2]
    cap = len(cellp) + (steps // 4 + 1) * inj
    grid = dict(ndim=3, n=n, dx=dx, dt=dt, window=True, window_speed=1.0)
    g = Sim(grid, C=list(TABLE1), precision=precision)
    sb = g.add_species(-1.0, Qb, len(beam_c))
    g.load_particles(sb, beam_c, beam_o, beam_u)
    sp = g.add_species(-1.0, Qp, cap)
    g.load_particles(sp, cellp, offp, up)
    g.set_injection(sp, (2, 2, 2), 1e-4, 77)
    g.set_sort_interval(5)
    o = OracleSim(n, dx, dt, C=TABLE1, window=True)
    o.add_particles(beam_c.astype(np.float64) + beam_o, beam_u, Qb, -1.0)
    o.add_particles(cellp.astype(np.float64) + offp, up, Qp, -1.0)
    o.set_injection((2, 2, 2), Qp, -1.0, 1e-4, 77)
    # the plasma occupies every (x2, x3) row of the window, so current is
    # deposited on every x1 line and the J1 correction covers the whole grid
    assert len(np.unique(cellp[:, 1] + n[1] * cellp[:, 2])) == n[1] * n[2]
    log("plasma whole grid %s: %d plasma + %d beam particles" % (precision, len(cellp), len(beam_c)))
    g.step(steps)
    o.step(steps)
    errs = field_errors(g, o)
    log("plasma whole grid %s fields: %s" % (precision, errs))
    assert max(errs.values()) < tol, errs
    xo, uo, ao = o.particles()
    nb = len(beam_c)
    xo, uo, ao = xo[nb:], uo[nb:], ao[nb:]
    c, of, uu, alive = g.particles(sp, cap)
    gid = g.last_ids[alive]
    assert np.array_equal(gid, np.flatnonzero(ao))
    dxm = float(np.abs((c[alive] + of[alive]) - xo[gid]).max())
    dum = float(np.abs(uu[alive] - uo[gid]).max() / np.abs(uo[gid]).max())
    log("plasma whole grid %s particles: max |dx| %.3g cells, max |du|/max |u| %.3g" % (precision, dxm, dum))
    assert dxm < ptol and dum < ptol
    g.close()
    o.close()
