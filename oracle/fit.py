"""App. C: customized axial stencil coefficients by constrained least squares
(TEST INFRASTRUCTURE ONLY).

With k1 normalized to k_g1 = 2 pi / dx1 (so k in [0, 1/2]) the customized
operator is  [k1]_p = sum_l C_l sin((2l-1) pi k) / pi  and the target is the
leapfrog time operator evaluated on the light line,
[k1]_t = kappa sin(pi k / kappa) / pi  (Sec. 3: [k]_1 = [k1]_t, kappa = dx1/dt).
The coefficients minimize  int_0^{1/2} w(k) ([k1]_p - [k1]_target)^2 dk
subject to  sum_j (2j-1)^{2i-1} / (2i-1)! C_j = delta_{i1},  i = 1..p/2
(App. C), solved through the KKT system [[A, M^T], [M, 0]] [C; lambda] = [b; e1]
with A_ij = (2/pi^2) int w sin((2i-1) pi k) sin((2j-1) pi k) dk and
b_i = (2/pi) int w sin((2i-1) pi k) [k1]_target dk, and the super-Gaussian
weight w = exp(-ln 2 (2k / w_k1)^n).

The paper leaves p, w_k1, n and the quadrature unstated.  Table 1 satisfies
only the first constraint row, so p = 2; w_k1 = 0.6, n = 10 reproduce it.
"""
import math

import numpy as np

# Table 1: C_1..C_16 for kappa = 4, r = 1 (quoted from the paper)
TABLE1 = np.array([
    1.248130933469396, -0.125139446419605, 0.040951412341664, -0.018181000724779,
    0.009121734802653, -0.004812019139855, 0.002570175265005, -0.001356670416082,
    0.000694723529383, -0.000339356036052, 0.000155316438379, -0.000065152281459,
    0.000024294488165, -0.000007666519708, 0.000001867004186, -0.000000273002422,
])


def target_e_with_yee_b(k, kappa):
    """[k]_E1 / k_g1 such that [k]_E1 [k]_B1 = [k1]_t^2 with [k]_B1 the Yee
    operator (Sec. 3: [k]_E1 != [k]_B1, product fixed), k normalized to k_g1:
    kappa^2 sin^2(pi k / kappa) / (pi sin(pi k)); the k -> 0 limit is k."""
    k = np.asarray(k, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = kappa ** 2 * np.sin(np.pi * k / kappa) ** 2 / (np.pi * np.sin(np.pi * k))
    return np.where(k == 0.0, 0.0, v)


def weight(k, wk1=0.6, nsg=10.0):
    return np.exp(-math.log(2.0) * (2.0 * k / wk1) ** nsg)


def target_time_operator(k, kappa):
    """[k1]_t / k_g1 on the light line, k normalized to k_g1."""
    return kappa * np.sin(np.pi * k / kappa) / np.pi


def constraint_matrix(M, p):
    rows = p // 2
    Mm = np.zeros((rows, M))
    for i in range(1, rows + 1):
        for j in range(1, M + 1):
            Mm[i - 1, j - 1] = (2 * j - 1) ** (2 * i - 1) / math.factorial(2 * i - 1)
    return Mm


def _nodes(nq, rule):
    if rule == "trapezoid":
        k = np.linspace(0.0, 0.5, nq + 1)
        w = np.full(nq + 1, 0.5 / nq)
        w[0] *= 0.5
        w[-1] *= 0.5
        return k, w
    if rule == "gauss":
        x, w = np.polynomial.legendre.leggauss(nq)
        return 0.25 * (x + 1.0), 0.25 * w
    raise ValueError(rule)


def fit_coefficients(kappa, M=16, p=2, wk1=0.6, nsg=10.0, nq=512, rule="trapezoid", target=None):
    """Solve the App. C KKT system; returns C[0..M-1]."""
    k, wq = _nodes(nq, rule)
    w = weight(k, wk1, nsg) * wq
    tgt = target_time_operator(k, kappa) if target is None else target(k)
    S = np.array([np.sin((2 * i - 1) * np.pi * k) for i in range(1, M + 1)])  # [M, nq]
    A = (2.0 / np.pi ** 2) * (S * w) @ S.T
    b = (2.0 / np.pi) * (S * w) @ tgt
    Mm = constraint_matrix(M, p)
    r = Mm.shape[0]
    K = np.zeros((M + r, M + r))
    K[:M, :M] = A
    K[:M, M:] = Mm.T
    K[M:, :M] = Mm
    rhs = np.concatenate([b, np.eye(r)[0] if r else np.zeros(0)])
    sol = np.linalg.solve(K, rhs)
    return sol[:M]


# ---- operator symbols (normalized: khat = k dx / 2 in [-pi/2, pi/2]) --------

def sym_yee(khat):
    """[k] dx/2 of the 2-point Yee difference (Eq. 14)."""
    return np.sin(khat)


def sym_custom(khat, C):
    """[k]_1 dx1/2 of the customized 2M-point operator (App. C)."""
    khat = np.asarray(khat, dtype=np.float64)
    out = np.zeros_like(khat)
    for l, c in enumerate(C, start=1):
        out = out + c * np.sin((2 * l - 1) * khat)
    return out


def sym_spectral(khat):
    """[k] dx/2 of the spectral operator (Eq. 20)."""
    return np.asarray(khat, dtype=np.float64)


def sym_time(khat, kappa):
    """[k1]_t dx1/2 on the light line: kappa sin(khat / kappa)."""
    return kappa * np.sin(np.asarray(khat, dtype=np.float64) / kappa)
