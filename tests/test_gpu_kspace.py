"""k-space field of a streaming charge in FP64 on the GPU (relpic_kspace_*)
against the CPU oracle's adaptive quadrature of the same integral, and the
self-forces the paper prints.

Tolerance: the integrand has integrable 1/sqrt(1 - A) singularities whose
positions are roots of A(k1) = 1 known only to FP64 rounding (delta ~ 1e-16);
any FP64 quadrature of such a point is then uncertain by about sqrt(delta),
i.e. ~1e-8 of the integral.  The two independent quadratures (tanh-sinh
panels on the GPU, adaptive Gauss-Kronrod on the CPU) are held to 1e-7."""
import numpy as np
import pytest

from gpu_common import log
from oracle import kspace
from oracle.fit import TABLE1

pytestmark = pytest.mark.gpu

I1 = np.array([-30, -21, -15, -10, -6, -3, -2, -1, 0, 1, 2, 4, 7, 10], dtype=np.float64)
TOL = 1e-7


def oracle_e1(solver, C, kappa, r, beta, order, tpow, nu_max):
    ks = kspace.KSpace(solver, kappa, r, order=order, beta=beta, C=C, tpow=tpow,
                       nus=tuple(range(-nu_max, nu_max + 1)))
    return ks.e1(I1)


@pytest.mark.parametrize("solver,kappa,r,beta,order,tpow", [
    ("yee", 4.0, 1.0, 1.0, 2, 0),
    ("yee", 4.0, 1.0, 1.0, 2, 1),
    ("yee", 4.0, 1.0, 1.0, 1, 0),
    ("yee", 2.5, 2.0, 1.0, 2, 1),
    ("yee", 4.0, 1.0, 0.9, 2, 0),
    ("custom", 4.0, 1.0, 1.0, 2, 0),
    ("custom", 4.0, 1.0, 1.0, 2, 2),
])
def test_e1_line_out_matches_oracle(solver, kappa, r, beta, order, tpow):
    from paper_1910_13529_amd.relpic import kspace_e1
    C = TABLE1 if solver == "custom" else None
    g = kspace_e1(I1, C=C, kappa=kappa, r=r, beta=beta, order=order, tpow=tpow, nu_max=1)
    o = oracle_e1(solver, C, kappa, r, beta, order, tpow, 1)
    err = np.abs(g - o).max() / np.abs(o).max()
    log("%s kappa=%g r=%g beta=%g p=%d q=%d: max |E1| %.4g, rel err %.3g" % (solver, kappa, r, beta, order, tpow,
                                                                             np.abs(o).max(), err))
    assert err < TOL


def test_self_forces_printed_and_oracle():
    from paper_1910_13529_amd.relpic import kspace_self_force
    lin = kspace_self_force(kappa=4.0, r=1.0, order=1, nu_max=0)
    quad = kspace_self_force(kappa=4.0, r=1.0, order=2, nu_max=0)
    # Sec. 2.2: -0.15 (linear), -0.10 (quadratic), zone nu = 0 of the Yee solver
    assert float("%.2g" % lin) == -0.15 and float("%.2g" % quad) == -0.10
    ol = kspace.KSpace("yee", 4.0, 1.0, order=1, nus=(0,)).self_force()
    oq = kspace.KSpace("yee", 4.0, 1.0, order=2, nus=(0,)).self_force()
    log("self-force linear %.12f (oracle %.12f), quadratic %.12f (oracle %.12f)" % (lin, ol, quad, oq))
    assert abs(lin - ol) < TOL * abs(ol) and abs(quad - oq) < TOL * abs(oq)
    # the aliased zones of the Yee solver carry no self-force at r = 1, kappa = 4
    alias = kspace_self_force(kappa=4.0, r=1.0, order=2, nu_max=1) - quad
    assert abs(alias) < 1e-12
    # customized (Table 1): F1 from the aliased zones only, as the oracle gives
    fc = kspace_self_force(C=TABLE1, kappa=4.0, r=1.0, order=2, nu_max=1)
    oc = kspace.KSpace("custom", 4.0, 1.0, order=2, C=TABLE1).self_force()
    log("customized self-force %.12g (oracle %.12g)" % (fc, oc))
    assert abs(fc - oc) < TOL * abs(oc)
