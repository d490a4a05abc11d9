"""Batched many-run path (relpic_batch_*): every run of a batch against the
same run stepped alone on the GPU, sampled runs against the FP64 CPU oracle,
and invariance of the results under tile shape, persistent grid, graph
recording and the autotuner.  Bar: FP64 within 1e-12 and FP32 within 1e-5
(relative to each component's maximum; see tests/gpu_common.py); field-only runs bit-identical
across tilings."""
import numpy as np
import pytest

from gpu_common import CANCEL_FRACTION, field_errors, log
from oracle.pic import OracleSim
from paper_1910_13529_amd import inputs, workloads

pytestmark = pytest.mark.gpu

FIELDS6 = ("E1", "E2", "E3", "B1", "B2", "B3")


def small_workload(nruns=6, seed=41, npart=1024, solver="mixed"):
    # ragged sizes: n1 and n2 not multiples of any tile edge in general
    return workloads.batch_workload(nruns, seed=seed, solver=solver, npart=npart, n1_range=(128, 300),
                                    n2_range=(12, 40))


def make_batch(runs, precision, with_particles=True):
    from paper_1910_13529_amd.relpic import Batch
    b = Batch([r["grid"] for r in runs], [r["C"] for r in runs], precision=precision)
    if with_particles:
        for br, r in zip(b.runs, runs):
            sid = br.add_species(-1.0, r["Q"], len(r["cell"]))
            br.load_particles(sid, r["cell"], r["offset"], r["u"])
    return b


def make_single(r, precision):
    from paper_1910_13529_amd.relpic import Sim
    s = Sim(r["grid"], C=r["C"], precision=precision)
    sid = s.add_species(-1.0, r["Q"], len(r["cell"]))
    s.load_particles(sid, r["cell"], r["offset"], r["u"])
    return s


def group_errors(a, b, names=FIELDS6):
    """per component max |a - b| over max |b| of that component, or over its
    field's (E or B) maximum when it is a cancelling component (below
    CANCEL_FRACTION of it); a component zero in b counts its absolute difference"""
    own = {n: float(np.abs(b[n]).max()) for n in names}
    group = {g: max(own[n] for n in names if n[0] == g) for g in "EB"}
    out = {}
    for n in names:
        sc = own[n] if own[n] >= CANCEL_FRACTION * group[n[0]] else group[n[0]]
        out[n] = float(np.abs(a[n] - b[n]).max()) / (sc or 1.0)
    return out


def fields_of(obj, names=FIELDS6):
    return {n: obj.field(n) for n in names}


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_batch_matches_single_runs(precision, tol):
    runs = small_workload()
    log("batch vs single, %s, %d runs, shapes 0/1/2, graph of 20 + 4 eager steps" % (precision, len(runs)))
    b = make_batch(runs, precision)
    b.set_tiling([k % 3 for k in range(len(runs))], 0)
    b.step(44)
    b.sync()
    for k, r in enumerate(runs):
        s = make_single(r, precision)
        s.step(44)
        s.sync()
        errs = group_errors(fields_of(b.runs[k]), fields_of(s))
        log("run %d (%s, n=%s): %s" % (k, "yee" if r["C"] is None else "custom", r["grid"]["n"][:2],
                                        max(errs.values())))
        assert max(errs.values()) < tol, (k, errs)
        cb, ob, ub, ab = b.runs[k].particles(0, len(r["cell"]))
        cs, os_, us, as_ = s.particles(0, len(r["cell"]))
        assert ab.all() and as_.all()
        xb = cb.astype(np.float64) + ob
        xs = cs.astype(np.float64) + os_
        assert np.abs(xb - xs).max() < (1e-12 if precision == "fp64" else 1e-4)
        assert (np.linalg.norm(ub - us, axis=1) / np.linalg.norm(us, axis=1)).max() < tol * 10
        assert b.runs[k].get_step()[0] == 44
        s.close()
    b.close()


def test_batch_vs_oracle_sampled_fp64():
    runs = small_workload()
    b = make_batch(runs, "fp64")
    b.step(30)
    b.sync()
    for k in (0, 1, 4):
        r = runs[k]
        log("batch run %d vs oracle (%s)" % (k, "yee" if r["C"] is None else "custom"))
        o = OracleSim(r["grid"]["n"][:2], r["grid"]["dx"][:2], r["grid"]["dt"],
                      C=[1.0] if r["C"] is None else list(r["C"]), window=False)
        o.add_particles(r["cell"].astype(np.float64) + r["offset"], r["u"], r["Q"], -1.0)
        o.step(30)
        errs = field_errors(b.runs[k], o)
        assert max(errs.values()) < 1e-12, (k, errs)
        o.close()
    b.close()


def test_batch_vs_oracle_sampled_fp32():
    runs = small_workload(seed=43)
    b = make_batch(runs, "fp32")
    b.step(30)
    b.sync()
    for k in (0, 3):
        r = runs[k]
        log("fp32 batch run %d vs fp64 oracle (%s)" % (k, "yee" if r["C"] is None else "custom"))
        o = OracleSim(r["grid"]["n"][:2], r["grid"]["dx"][:2], r["grid"]["dt"],
                      C=[1.0] if r["C"] is None else list(r["C"]), window=False)
        o.add_particles(r["cell"].astype(np.float64) + r["offset"], r["u"], r["Q"], -1.0)
        o.step(30)
        errs = field_errors(b.runs[k], o)
        assert max(errs.values()) < 1e-5, (k, errs)
        o.close()
    b.close()


def seeded_fields(b, runs, seed):
    for k, (br, r) in enumerate(zip(b.runs, runs)):
        shape = (r["grid"]["n"][1], r["grid"]["n"][0])
        for name, arr in zip(FIELDS6, inputs.random_fields(seed + k, shape)):
            br.set_field(name, arr)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_field_only_bitwise_across_tilings(precision):
    runs = small_workload(nruns=5, seed=47)
    configs = [([0] * 5, 0, 20), ([2] * 5, 16, 0), ([1] * 5, 0, 2), ([0, 1, 2, 1, 0], 8, 20)]
    results = []
    for shapes, grid, G in configs:
        log("field-only %s: shapes %s grid %d graph %d" % (precision, shapes, grid, G))
        b = make_batch(runs, precision, with_particles=False)
        seeded_fields(b, runs, 900)
        b.set_tiling(shapes, grid)
        b.set_graph_steps(G)
        b.step(22)
        b.sync()
        results.append([fields_of(br) for br in b.runs])
        b.close()
    for res in results[1:]:
        for k in range(len(runs)):
            for n in FIELDS6:
                assert np.array_equal(res[k][n], results[0][k][n]), (k, n)
    # and the same as each run alone
    from paper_1910_13529_amd.relpic import Sim
    for k, r in enumerate(runs):
        s = Sim(r["grid"], C=r["C"], precision=precision)
        shape = (r["grid"]["n"][1], r["grid"]["n"][0])
        for name, arr in zip(FIELDS6, inputs.random_fields(900 + k, shape)):
            s.set_field(name, arr)
        s.step(22)
        f = fields_of(s)
        for n in FIELDS6:
            assert np.array_equal(f[n], results[0][k][n]), (k, n)
        s.close()


def test_autotune_keeps_state_and_results():
    runs = small_workload(nruns=6, seed=53)
    b = make_batch(runs, "fp64")
    b.step(3)
    before = [fields_of(br) for br in b.runs]
    rep = b.autotune(reps=3)
    log("autotune: %s" % rep)
    after = [fields_of(br) for br in b.runs]
    for k in range(len(runs)):
        for n in FIELDS6:
            assert np.array_equal(before[k][n], after[k][n])
    assert 0 <= rep["choice"] <= 3 and rep["ms_chosen"] > 0
    assert sum(rep["runs_per_shape"]) == len(runs)
    shapes, grid = b.tiling()
    assert grid % 8 == 0 and all(0 <= v < 3 for v in shapes)
    b.step(17)
    ref = make_batch(runs, "fp64")
    ref.step(20)
    for k in range(len(runs)):
        errs = group_errors(fields_of(b.runs[k]), fields_of(ref.runs[k]))
        assert max(errs.values()) < 1e-12, (k, errs)
    b.close()
    ref.close()


def test_run_stepped_alone_inside_batch():
    """A run handle stepped on its own between batch steps: the batch rebuilds
    its tables and every run still matches a lone simulation."""
    runs = small_workload(nruns=3, seed=59)
    b = make_batch(runs, "fp64")
    b.step(5)
    b.runs[0].step(3)
    b.step(5)
    b.sync()
    for k, extra in ((0, 3), (1, 0), (2, 0)):
        s = make_single(runs[k], "fp64")
        s.step(10 + extra)
        errs = group_errors(fields_of(b.runs[k]), fields_of(s))
        assert max(errs.values()) < 1e-12, (k, errs)
        assert b.runs[k].get_step()[0] == 10 + extra
        s.close()
    b.close()


def test_full_batched_workload_sampled():
    """The 256-run workload (23.6 M cells, 1.05 M particles) in FP32, in the
    launch configuration the benchmark times: sampled runs against the same
    run alone, every run's diagnostics sane."""
    runs = workloads.batch_workload(256)
    log("full batched workload: %d cells" % sum(r["grid"]["n"][0] * r["grid"]["n"][1] for r in runs))
    b = make_batch(runs, "fp32")
    b.autotune(reps=3)
    sample = range(0, 256, 15)
    # fields start at zero, so div E - rho = -rho(0) at every later time if
    # the deposit conserves charge: the residual's maximum stays max |rho(0)|
    d0 = {k: b.runs[k].diagnostics() for k in sample}
    b.step(40)
    b.sync()
    for k in (0, 77, 154, 255):
        s = make_single(runs[k], "fp32")
        s.step(40)
        errs = group_errors(fields_of(b.runs[k]), fields_of(s))
        log("run %d: %g" % (k, max(errs.values())))
        assert max(errs.values()) < 1e-5, (k, errs)
        s.close()
    for k in sample:
        d = b.runs[k].diagnostics()
        assert d["error_word"] == 0 and d["n_alive"] == 4096 and d["step"] == 40
        assert np.isfinite(d["w_field"]) and d["w_field"] > 0
        assert abs(d["charge"] - d0[k]["charge"]) < 1e-6 * abs(d0[k]["charge"])
        r0 = d0[k]["rho_max"]
        assert abs(d["gauss_max"] - r0) < 1e-4 * r0, (k, d, r0)
    b.close()
