"""Pins of the App. C coefficient fit and the operator symbols against Table 1
and the mathematics of the customized operator."""
import math

import numpy as np
import pytest

from oracle import fit


def test_table1_constraint_rows_fix_order_p2():
    # Table 1 meets the consistency row i = 1 (sum (2j-1) C_j = 1) to round-off
    # and misses row i = 2, so the fit was run with p = 2.
    rows = fit.constraint_matrix(16, 8) @ fit.TABLE1
    assert abs(rows[0] - 1.0) < 1e-14
    assert abs(rows[1]) > 1e-3


@pytest.mark.parametrize("rule,nq,tol", [("trapezoid", 512, 1e-6), ("trapezoid", 2048, 2e-7),
                                         ("gauss", 4000, 1e-6)])
def test_fit_reproduces_table1(rule, nq, tol):
    C = fit.fit_coefficients(4.0, M=16, p=2, wk1=0.6, nsg=10.0, nq=nq, rule=rule)
    assert np.abs(C - fit.TABLE1).max() < tol


def test_fit_constraint_holds_other_kappa():
    for kappa in (2.5, 3.0, 6.0, 10.0):
        C = fit.fit_coefficients(kappa, M=12)
        assert abs(np.sum((2 * np.arange(1, 13) - 1) * C) - 1.0) < 1e-12


def test_table1_symbol_matches_time_operator():
    # [k]_1 of Table 1 tracks [k1]_t = kappa sin(khat/kappa) (Fig. 5 upper left):
    # tight at low k, a few per cent below at the Nyquist edge.
    kh = np.linspace(1e-3, math.pi / 2, 4001)
    rel = (fit.sym_custom(kh, fit.TABLE1) - fit.sym_time(kh, 4.0)) / fit.sym_time(kh, 4.0)
    assert np.abs(rel[kh <= 1.0]).max() < 2e-7
    assert -0.06 < rel[-1] < -0.04


def test_yee_is_m1_custom():
    kh = np.linspace(-1.5, 1.5, 101)
    assert np.allclose(fit.sym_custom(kh, [1.0]), fit.sym_yee(kh), atol=0, rtol=0)


def test_custom_symbol_small_k_is_consistent():
    # with sum (2l-1) C_l = 1 the operator is a consistent first derivative
    kh = 1e-5
    assert abs(fit.sym_custom(kh, fit.TABLE1) / kh - 1.0) < 1e-9
