"""The paper's k-space field of a charge streaming along x1 on the grid
(TEST INFRASTRUCTURE ONLY).

Sec. 2 expresses the on-axis axial field of a point charge q moving at beta
along x1 on a 2D grid as a k-space integral (Eq. 13; general beta through
Eqs. 8-9 and the aliased density of App. A):

  E1(i1', i2=0) = -(q/(2 pi)^2) int dk1 (i/[k]_B1) sum_nu S1(k1 + nu k_g1)
                   * I_nu(k1) exp(i k1 dx1 (i1' + 1/2)),
  I_nu(k1) = int_{-k_g2/2}^{k_g2/2} dk2 T(k2) X / (X - [k]_E2 [k]_B2),
  X = [beta (k1 + nu k_g1)]_t^2 - [k]_E1 [k]_B1,

with i1' the E1 index relative to the particle (E1 sits at i1 + 1/2), the
particle on a node, and T the transverse density factor of the deposit
(T = 1 for the paper's linear transverse shape, whose aliases sum to 1; the
quadratic spline sampled at a node gives T = 1 - sin^2(k2 dx2/2)/2).

In normalized variables khat = k1 dx1/2, theta = k2 dx2/2, r = dx2/dx1,
kappa = dx1/dt this becomes

  E1 dx1 / q = -(1/(2 pi^2 r)) int_{-pi/2}^{pi/2} dkhat (i/sigmaB(khat))
               sum_nu Shat(khat + nu pi) Ihat_nu(khat) exp(i khat (2 i1' + 1))

with sigmaE = [k]_E1 dx1/2, sigmaB = [k]_B1 dx1/2 (equal unless the operators
on E and on B differ, Sec. 3), Ihat = int dtheta T A/(A - sigma2(theta)^2),
A = r^2 (tau^2 - sigmaE sigmaB), tau = kappa sin(beta (khat + nu pi)/kappa).

The k2 integral is done in closed form (App. D, with the typo 1-A^2 read as
1-A).  Poles (0 < A < 1 for the Yee transverse operator, 0 < A < pi^2/4 for
the spectral one) take the causal prescription omega -> omega + i0, i.e.
A -> A + i0 s with s = sign(sin(beta k1' dt)) (App. D states it for nu = 0:
k1 > 0 gives -i pi sqrt(A/(1-A))).  The k1 integral is adaptive quadrature
with breakpoints at every region boundary.

Off axis (E1 at transverse node i2, Yee transverse operator) the theta
integral carries cos(2 i2 theta) and is done in closed form by residues
(k2_integral_n).  In 3D (KSpace3D) the x3 integral is that closed form and
the x2 integral is adaptive quadrature, nested inside the k1 quadrature.
"""
import math

import numpy as np
from scipy import integrate, optimize

from .fit import sym_custom, sym_spectral, sym_yee


def shape_hat(khat, order):
    """Fourier transform of the order-p B-spline: sinc(khat)^(p+1)."""
    khat = np.asarray(khat, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(khat == 0.0, 1.0, np.sin(khat) / np.where(khat == 0.0, 1.0, khat))
    return s ** (order + 1)


def axial_symbol(solver, C=None, kappa=None):
    if solver == "yee":
        return sym_yee
    if solver == "spectral":
        return sym_spectral
    if solver == "custom":
        Cc = np.asarray(C, dtype=np.float64)
        return lambda k: sym_custom(k, Cc)
    if solver == "exact":  # [k]_1 = [k1]_t exactly (Sec. 3)
        return lambda k: kappa * np.sin(np.asarray(k, dtype=np.float64) / kappa)
    raise ValueError(solver)


def transverse_kind(solver):
    return "spectral" if solver == "spectral" else "yee"


def k2_integral(A, s, kind="yee", tpow=0):
    """Ihat(A) = int_{-pi/2}^{pi/2} dtheta T^tpow A / (A + i0 s - sigma2^2)."""
    if A == 0.0:
        return 0.0 + 0.0j
    if kind == "yee":
        if A < 0.0 or A > 1.0:
            base = math.pi * math.sqrt(-A / (1.0 - A)) + 0.0j
        else:
            base = -1j * s * math.pi * math.sqrt(A / (1.0 - A))
        if tpow == 0:
            return base
        h = 1.0 - 0.5 * A
        if tpow == 1:
            return h * base + 0.5 * math.pi * A
        if tpow == 2:
            return h * h * base + h * math.pi * A + 0.25 * A * (math.pi * A - 0.5 * math.pi)
        raise ValueError(tpow)
    if kind == "spectral":
        if tpow != 0:
            raise ValueError("spectral transverse operator: only T = 1")
        if A < 0.0:
            a = -A
            return 2.0 * math.sqrt(a) * math.atan(math.pi / (2.0 * math.sqrt(a))) + 0.0j
        rA = math.sqrt(A)
        if A > math.pi ** 2 / 4.0:
            return 2.0 * rA * math.atanh(math.pi / (2.0 * rA)) + 0.0j
        return 2.0 * rA * math.atanh(2.0 * rA / math.pi) - 1j * s * math.pi * rA
    raise ValueError(kind)


def k2_integral_n(A, s, tpow=0, n=0):
    """Ihat_n(A) = int_{-pi/2}^{pi/2} dtheta T^tpow A cos(2 n theta) / (A + i0 s - sin^2 theta)
    for the Yee transverse operator (E1 at transverse node n; T = 1 - sin^2/2).

    With phi = 2 theta the denominator is (a + cos phi)/2, a = 2A - 1, and
    the residue at the root z of z^2 + 2 a z + 1 inside the unit circle gives
      int_{-pi}^{pi} cos(n phi) / (a + cos phi) dphi = 2 pi z^|n| / w,  z = w - a,
    with w = sqrt(a^2 - 1) of the sign of a when |a| > 1 and, on the pole
    (|a| < 1), w = i s sqrt(1 - a^2): the causal shift a -> a + i0 s moves the
    root z = -a + i s sqrt(1 - a^2) inside.  T = (3 + cos phi)/4 is divided out:
      T / (a + c)   = (1/4)  [1 + (3 - a) / (a + c)],
      T^2 / (a + c) = (1/16) [(a + c) + 2 (3 - a) + (3 - a)^2 / (a + c)],  c = cos phi,
    whose polynomial parts integrate against cos(n phi) to 2 pi [n = 0] and
    pi [n = 1]."""
    n = abs(int(n))
    if A == 0.0:
        return 0.0 + 0.0j
    a = 2.0 * A - 1.0
    if abs(a) > 1.0:
        w = complex(math.copysign(math.sqrt(a * a - 1.0), a), 0.0)
    else:
        w = 1j * s * math.sqrt(1.0 - a * a)
    if w == 0.0:  # A = 0 or 1 exactly: an integrable end singularity, measure zero
        return 0.0 + 0.0j
    z = w - a
    In = 2.0 * math.pi * z ** n / w
    d0 = 2.0 * math.pi if n == 0 else 0.0
    d1 = math.pi if n == 1 else 0.0
    if tpow == 0:
        J = In
    elif tpow == 1:
        J = 0.25 * (d0 + (3.0 - a) * In)
    elif tpow == 2:
        J = (a * d0 + d1 + 2.0 * (3.0 - a) * d0 + (3.0 - a) ** 2 * In) / 16.0
    else:
        raise ValueError(tpow)
    return A * J


class KSpace:
    """E1 and self-force of a streaming point charge (2D), on axis or at
    transverse node i2."""

    def __init__(self, solver="yee", kappa=4.0, r=1.0, order=2, beta=1.0, C=None, tpow=0, nus=(-1, 0, 1), CB=None,
                 filt=None):
        """solver names the operator on E (symbol [k]_E1); CB, when given,
        the customized operator on B ([k]_B1, Sec. 3 allows them to differ),
        else [k]_B1 = [k]_E1.  filt = (n, c): the current is smoothed along
        x1 by n binomial (1, 2, 1)/4 passes and one compensator pass of
        symbol 1 + c sin^2(k1 dx1/2), so the source carries the factor
        cos^(2n)(khat) (1 + c sin^2 khat) of the grid wavenumber khat."""
        self.solver = solver
        self.kappa = float(kappa)
        self.r = float(r)
        self.order = order
        self.beta = float(beta)
        self.sigma1 = axial_symbol(solver, C, kappa)
        self.sigmaB = self.sigma1 if CB is None else axial_symbol("custom", CB, kappa)
        self.filt = filt
        self.kind = transverse_kind(solver)
        self.tpow = tpow
        self.nus = tuple(nus)

    def filter_factor(self, kh):
        if self.filt is None:
            return 1.0
        n, c = self.filt
        return math.cos(kh) ** (2 * n) * (1.0 + c * math.sin(kh) ** 2)

    # X dx1^2/4 on zone nu
    def xhat(self, kh, nu):
        tau = self.kappa * np.sin(self.beta * (kh + nu * np.pi) / self.kappa)
        return tau * tau - self.sigma1(kh) * self.sigmaB(kh)

    def A(self, kh, nu):
        return self.r ** 2 * self.xhat(kh, nu)

    def sgn(self, kh, nu):
        v = math.sin(2.0 * self.beta * (kh + nu * math.pi) / self.kappa)
        return 1.0 if v > 0 else (-1.0 if v < 0 else 0.0)

    def ihat(self, kh, nu, i2=0):
        if i2 == 0:
            return k2_integral(float(self.A(kh, nu)), self.sgn(kh, nu), self.kind, self.tpow)
        if self.kind != "yee":
            raise ValueError("off-axis fields: Yee transverse operator only")
        return k2_integral_n(float(self.A(kh, nu)), self.sgn(kh, nu), self.tpow, i2)

    def breakpoints(self, nu, ngrid=4001):
        """khat where A = 0, A = 1 (Yee) or A = pi^2/4 (spectral), sin(beta k1' dt) = 0, and 0."""
        kh = np.linspace(-np.pi / 2, np.pi / 2, ngrid)
        pts = {0.0}
        levels = [0.0, 1.0] if self.kind == "yee" else [0.0, np.pi ** 2 / 4.0]
        for lev in levels:
            f = lambda k, lev=lev: float(self.A(k, nu)) - lev
            v = np.array([f(k) for k in kh])
            for i in range(len(kh) - 1):
                if v[i] == 0.0:
                    pts.add(float(kh[i]))
                elif v[i] * v[i + 1] < 0.0:
                    pts.add(float(optimize.brentq(f, kh[i], kh[i + 1], xtol=1e-15)))
        g = lambda k: math.sin(2.0 * self.beta * (k + nu * math.pi) / self.kappa)
        v = np.array([g(k) for k in kh])
        for i in range(len(kh) - 1):
            if v[i] * v[i + 1] < 0.0:
                pts.add(float(optimize.brentq(g, kh[i], kh[i + 1], xtol=1e-15)))
        pts = sorted(p for p in pts if -np.pi / 2 < p < np.pi / 2)
        return [-np.pi / 2] + pts + [np.pi / 2]

    def _integrate(self, fn, nu):
        bp = self.breakpoints(nu)
        total = 0.0
        for a, b in zip(bp[:-1], bp[1:]):
            if b - a < 1e-14:
                continue
            v, _ = integrate.quad(fn, a, b, limit=400, epsabs=1e-14, epsrel=1e-11)
            total += v
        return total

    def e1(self, i1rel, i2=0):
        """E1 dx1 / q at E1 index i1' relative to the particle, on the x2 row
        i2 rows from the particle's (E1 at (i1' + 1/2, i2))."""
        out = []
        for ip in np.atleast_1d(i1rel):
            ph = 2.0 * float(ip) + 1.0
            tot = 0.0
            for nu in self.nus:
                def fn(kh, nu=nu):
                    s1 = float(self.sigmaB(kh))  # i / [k]_B1 (continuity with the B operator)
                    if s1 == 0.0:
                        return 0.0
                    val = (1j / s1) * float(shape_hat(kh + nu * np.pi, self.order)) * self.ihat(kh, nu, i2)
                    val = val * self.filter_factor(kh)
                    return (val * complex(math.cos(ph * kh), math.sin(ph * kh))).real
                tot += self._integrate(fn, nu)
            out.append(-tot / (2.0 * np.pi ** 2 * self.r))
        return np.array(out)

    def self_force(self, gather_order=None):
        """F1 dx1 / q^2 in the paper's convention (Eqs. 19, 25): the k1-space
        field weighted by the unaliased gather shape S(k1), no staggering phase."""
        go = self.order if gather_order is None else gather_order
        tot = 0.0
        for nu in self.nus:
            def fn(kh, nu=nu):
                s1 = float(self.sigmaB(kh))
                if s1 == 0.0:
                    return 0.0
                val = (1j / s1) * float(shape_hat(kh, go)) * float(shape_hat(kh + nu * np.pi, self.order)) * self.ihat(kh, nu)
                return (val * self.filter_factor(kh)).real
            tot += self._integrate(fn, nu)
        return -tot / (2.0 * np.pi ** 2 * self.r)


    def lattice_self_force(self, gather_order=2):
        """F1 dx1 / q^2 as a PIC code measures it: the on-axis E1 line-out at
        the E1 points (i1' + 1/2) around a particle on a node, interpolated to
        the particle with the B-spline of order gather_order along x1 (the
        gather's aliases included).  The transverse gather enters through
        tpow (tpow = 2: quadratic deposit and quadratic gather in x2)."""
        ip = np.arange(-3, 3)
        w = bspline(ip + 0.5, gather_order)
        keep = w != 0.0
        return float(np.dot(w[keep], self.e1(ip[keep])))


class KSpace3D:
    """E1 of a point charge streaming along x1 on a 3D grid (Eq. 9 with the
    x2 and x3 integrals), at the E1 point (i1' + 1/2, i2, i3) relative to
    the particle on a node, Yee transverse operators, r2 = dx2/dx1,
    r3 = dx3/dx1:

      E1 dx1^2 / q = -(1/(2 pi^3 r2 r3)) sum_nu int dkhat
                      Re[(i/sigmaB) Shat(khat + nu pi) I3 e^{i khat (2 i1' + 1)}],
      I3 = int dtheta2 dtheta3 T2 T3 X / (X - sin^2 theta2 / r2^2 - sin^2 theta3 / r3^2)
           cos(2 i2 theta2) cos(2 i3 theta3),

    X = tau^2 - sigmaE sigmaB (X dx1^2/4 of the 2D case, with the causal
    shift X -> X + i0 s), T = (1 - sin^2/2)^tpow per transverse direction.
    The theta3 integral is k2_integral_n at A3 = r3^2 (X - sin^2 theta2 /
    r2^2) divided by A3: I3 = r3^2 X int dtheta2 T2 cos(2 i2 theta2)
    J(A3) with J = k2_integral_n / A.  The theta2 integral is adaptive
    quadrature split where A3 crosses 0 and 1."""

    def __init__(self, solver="yee", kappa=4.0, r2=1.0, r3=1.0, order=2, beta=1.0, C=None, tpow=0, nus=(-1, 0, 1),
                 CB=None):
        self.kappa = float(kappa)
        self.r2 = float(r2)
        self.r3 = float(r3)
        self.order = order
        self.beta = float(beta)
        self.sigma1 = axial_symbol(solver, C, kappa)
        self.sigmaB = self.sigma1 if CB is None else axial_symbol("custom", CB, kappa)
        if transverse_kind(solver) != "yee":
            raise ValueError("3D: Yee transverse operators only")
        self.tpow = tpow
        self.nus = tuple(nus)

    def xhat(self, kh, nu):
        tau = self.kappa * math.sin(self.beta * (kh + nu * math.pi) / self.kappa)
        return tau * tau - float(self.sigma1(kh)) * float(self.sigmaB(kh))

    def sgn(self, kh, nu):
        v = math.sin(2.0 * self.beta * (kh + nu * math.pi) / self.kappa)
        return 1.0 if v > 0 else (-1.0 if v < 0 else 0.0)

    def i3(self, kh, nu, i2, i3):
        X = self.xhat(kh, nu)
        if X == 0.0:
            return 0.0 + 0.0j
        s = self.sgn(kh, nu)
        r2, r3, p = self.r2, self.r3, self.tpow

        def f(t2):
            A3 = r3 * r3 * (X - math.sin(t2) ** 2 / (r2 * r2))
            if A3 == 0.0:
                return 0.0 + 0.0j
            T2 = (1.0 - 0.5 * math.sin(t2) ** 2) ** p
            return T2 * math.cos(2.0 * i2 * t2) * k2_integral_n(A3, s, p, i3) / A3

        # A3 = 0 at sin^2 t2 = r2^2 X, A3 = 1 at sin^2 t2 = r2^2 (X - 1/r3^2); the integrand is even in t2
        pts = [0.0, math.pi / 2]
        for v in (r2 * r2 * X, r2 * r2 * (X - 1.0 / (r3 * r3))):
            if 0.0 < v < 1.0:
                pts.append(math.asin(math.sqrt(v)))
        pts = sorted(pts)
        re = im = 0.0
        for a, b in zip(pts[:-1], pts[1:]):
            if b - a < 1e-15:
                continue
            re += integrate.quad(lambda t: f(t).real, a, b, limit=200, epsabs=1e-13, epsrel=1e-11)[0]
            im += integrate.quad(lambda t: f(t).imag, a, b, limit=200, epsabs=1e-13, epsrel=1e-11)[0]
        return 2.0 * r3 * r3 * X * complex(re, im)

    def breakpoints(self, nu, ngrid=2001):
        """khat where X crosses 0, 1/r3^2, 1/r2^2, 1/r2^2 + 1/r3^2 (where the
        theta2 integrand changes form), sin(beta k1' dt) = 0, and 0."""
        kh = np.linspace(-np.pi / 2, np.pi / 2, ngrid)
        pts = {0.0}
        levels = [0.0, 1.0 / self.r3 ** 2, 1.0 / self.r2 ** 2, 1.0 / self.r2 ** 2 + 1.0 / self.r3 ** 2]
        for lev in levels:
            f = lambda k, lev=lev: self.xhat(k, nu) - lev
            v = np.array([f(k) for k in kh])
            for i in range(len(kh) - 1):
                if v[i] == 0.0:
                    pts.add(float(kh[i]))
                elif v[i] * v[i + 1] < 0.0:
                    pts.add(float(optimize.brentq(f, kh[i], kh[i + 1], xtol=1e-15)))
        g = lambda k: math.sin(2.0 * self.beta * (k + nu * math.pi) / self.kappa)
        v = np.array([g(k) for k in kh])
        for i in range(len(kh) - 1):
            if v[i] * v[i + 1] < 0.0:
                pts.add(float(optimize.brentq(g, kh[i], kh[i + 1], xtol=1e-15)))
        pts = sorted(p for p in pts if -np.pi / 2 < p < np.pi / 2)
        return [-np.pi / 2] + pts + [np.pi / 2]

    def e1(self, i1rel, i2=0, i3=0, epsrel=1e-9):
        """E1 dx1^2 / q at (i1' + 1/2, i2, i3) relative to the particle."""
        out = []
        for ip in np.atleast_1d(i1rel):
            ph = 2.0 * float(ip) + 1.0
            tot = 0.0
            for nu in self.nus:
                def fn(kh, nu=nu):
                    sB = float(self.sigmaB(kh))
                    if sB == 0.0:
                        return 0.0
                    val = (1j / sB) * float(shape_hat(kh + nu * np.pi, self.order)) * self.i3(kh, nu, i2, i3)
                    return (val * complex(math.cos(ph * kh), math.sin(ph * kh))).real
                bp = self.breakpoints(nu)
                for a, b in zip(bp[:-1], bp[1:]):
                    if b - a < 1e-14:
                        continue
                    tot += integrate.quad(fn, a, b, limit=200, epsabs=1e-13, epsrel=epsrel)[0]
            out.append(-tot / (2.0 * math.pi ** 3 * self.r2 * self.r3))
        return np.array(out)


def bspline(d, order):
    """Centred B-spline of order 1 (hat) or 2 (quadratic) at distances d (cells)."""
    d = np.abs(np.asarray(d, dtype=np.float64))
    if order == 1:
        return np.where(d < 1.0, 1.0 - d, 0.0)
    if order == 2:
        return np.where(d <= 0.5, 0.75 - d * d, np.where(d < 1.5, 0.5 * (1.5 - d) ** 2, 0.0))
    raise ValueError(order)


# ---- regime thresholds (Sec. 2.2, 2.3, 3) ----------------------------------

def r_crit():
    """Yee, nu = 0: above this r a space-charge zone can appear (Sec. 2.2)."""
    return 2.0 / math.sqrt(math.pi ** 2 - 4.0)


def kappa_r_yee(r):
    """kappa_r^2 sin^2(pi / (2 kappa_r)) = 1 + r^-2 (Sec. 2.2)."""
    f = lambda k: k * k * math.sin(math.pi / (2.0 * k)) ** 2 - (1.0 + r ** -2)
    return optimize.brentq(f, 1.0 + 1e-12, 100.0, xtol=1e-15)


def kappa_r_spectral():
    """kappa_r^2 sin^2(3 pi / (2 kappa_r)) = pi^2 / 2, r = 1 (Sec. 2.3)."""
    f = lambda k: k * k * math.sin(1.5 * math.pi / k) ** 2 - math.pi ** 2 / 2.0
    return optimize.brentq(f, 1.6, 10.0, xtol=1e-15)


def kappa_r_custom():
    """sin^2(3 pi / (2 kappa_r)) - sin^2(pi / (2 kappa_r)) = 1 / kappa_r^2 (Sec. 3)."""
    f = lambda k: math.sin(1.5 * math.pi / k) ** 2 - math.sin(0.5 * math.pi / k) ** 2 - 1.0 / k ** 2
    return optimize.brentq(f, 1.6, 10.0, xtol=1e-15)


def regime_nu0(ks, ngrid=20001):
    """Classify zone nu = 0 from the symbols alone: 'cerenkov' if 0 < A < 1
    for every khat in (0, pi/2], 'space-charge' if never, else 'mixed'."""
    kh = np.linspace(1e-6, np.pi / 2, ngrid)
    A = ks.A(kh, 0)
    if ks.kind == "yee":
        pole = (A > 0.0) & (A < 1.0)
    else:
        pole = (A > 0.0) & (A < np.pi ** 2 / 4.0)
    if pole.all():
        return "cerenkov"
    if not pole.any():
        return "space-charge"
    return "mixed"
