"""The allocation-free k-space entry point (relpic_kspace_e1_noalloc) against
relpic_kspace_e1, through the C ABI: two calls in a row, the second with
fewer points, and the size limits."""
import ctypes

import numpy as np
import pytest

from oracle.fit import TABLE1

pytestmark = pytest.mark.gpu


def _call(L, relpic, fn, q, pts):
    x = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.full(x.size, np.nan)
    st = getattr(L, fn)(ctypes.byref(q), None, x.size, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return st, out


@pytest.mark.parametrize("solver", ["yee", "custom"])
def test_noalloc_matches_allocating_entry_point(solver):
    from paper_1910_13529_amd import relpic
    L = relpic.load()
    C = None if solver == "yee" else TABLE1
    q, keep = relpic._kspace_struct(C, 4.0, 1.0, 1.0, 2, 1, 2)
    big = np.arange(-40, 24, dtype=np.float64)
    small = np.array([-3.0, 0.0, 5.0])
    for pts in (big, small):  # the second call is smaller: stale scratch must not leak into it
        st_a, ref = _call(L, relpic, "relpic_kspace_e1", q, pts)
        st_b, got = _call(L, relpic, "relpic_kspace_e1_noalloc", q, pts)
        assert st_a == relpic.RELPIC_OK and st_b == relpic.RELPIC_OK, L.relpic_last_error()
        assert np.all(np.isfinite(got))
        # same panels, same kernel: identical up to summation order (none here)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (pts, got, ref)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_1910_13529_amd import relpic
    L = relpic.load()
    q, keep = relpic._kspace_struct(None, 4.0, 1.0, 1.0, 2, 0, 1)
    st, _ = _call(L, relpic, "relpic_kspace_e1_noalloc", q, np.zeros(4097))
    assert st == relpic.RELPIC_EINVAL
    assert b"4096" in L.relpic_last_error()
    # and a valid call right after still works
    st, out = _call(L, relpic, "relpic_kspace_e1_noalloc", q, np.array([0.0, 1.0]))
    assert st == relpic.RELPIC_OK and np.all(np.isfinite(out))
