"""ctypes front end of the plain-C FP64 PIC oracle (TEST INFRASTRUCTURE ONLY).

The arithmetic lives in pic_oracle.c; this module only builds the shared
library with gcc, marshals numpy arrays and names the field components.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "liboracle_pic.so")

FIELDS = ("E1", "E2", "E3", "B1", "B2", "B3", "J1", "J2", "J3")

_lib = None


def build(force=False):
    """Compile pic_oracle.c with gcc -O2 (OpenMP on) into liboracle_pic.so."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        Lg = ctypes.c_long
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_create.restype = P
        L.orc_create.argtypes = [ctypes.c_int, lp, dp, D, ctypes.c_int, D, ctypes.c_int, dp, ctypes.c_int, dp,
                                 ctypes.c_int]
        L.orc_destroy.argtypes = [P]
        L.orc_add_particles.restype = Lg
        L.orc_add_particles.argtypes = [P, Lg, dp, dp, D, D]
        L.orc_step.argtypes = [P, Lg]
        L.orc_field_only.argtypes = [P, Lg]
        L.orc_get_field.argtypes = [P, ctypes.c_int, dp]
        L.orc_set_field.argtypes = [P, ctypes.c_int, dp]
        L.orc_num_particles.restype = Lg
        L.orc_num_particles.argtypes = [P]
        L.orc_window_start.restype = Lg
        L.orc_window_start.argtypes = [P]
        L.orc_steps_done.restype = Lg
        L.orc_steps_done.argtypes = [P]
        L.orc_correction_halfwidth.restype = Lg
        L.orc_correction_halfwidth.argtypes = [P]
        L.orc_get_particles.argtypes = [P, dp, dp, ip]
        L.orc_rho.argtypes = [P, dp]
        L.orc_div_e.argtypes = [P, dp]
        L.orc_energy.argtypes = [P, dp, dp]
        L.orc_gather_at.argtypes = [P, Lg, dp, dp]
        L.orc_boris.argtypes = [D, D, dp, dp]
        L.orc_deposit_one.argtypes = [P, D, dp, dp, D]
        L.orc_correct_j1.argtypes = [P]
        L.orc_set_injection.argtypes = [P, ip, D, D, D, ctypes.c_uint64]
        L.orc_set_filter.argtypes = [P, ctypes.c_int, D]
        L.orc_filter_j.argtypes = [P]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleSim:
    """One FP64 PIC run on the CPU.

    n, dx: per-dimension cells and spacing (len = ndim); dt: time step;
    window: False = periodic x1, True = moving window at speed vwin;
    C: axial stencil coefficients of d+ (E -> B) and, unless CB is given, of
    d- (B -> E) as well (C = [1.0] is Yee); CB: coefficients of d- when the
    two differ (Sec. 3, [k]_E1 != [k]_B1); correct: apply the J1 correction
    (defaults to True whenever d- is not Yee).
    """

    def __init__(self, n, dx, dt, C=(1.0,), window=False, vwin=1.0, correct=None, CB=None):
        self.ndim = len(n)
        self.n = tuple(int(v) for v in n)
        self.shape = tuple(reversed(self.n))  # numpy view: [i3][i2][i1]
        C = np.ascontiguousarray(C, dtype=np.float64)
        CBa = np.ascontiguousarray(C if CB is None else CB, dtype=np.float64)
        if correct is None:
            # a d- stencil wider than two points (trailing zeros aside) needs it
            correct = int(np.flatnonzero(CBa).max(initial=0)) > 0
        nn = (ctypes.c_long * 3)(*(list(self.n) + [1] * (3 - self.ndim)))
        dd = np.ascontiguousarray(list(dx) + [1.0] * (3 - self.ndim), dtype=np.float64)
        self._h = lib().orc_create(self.ndim, nn, _dp(dd), float(dt), int(bool(window)), float(vwin),
                                   len(C), _dp(C), 0 if CB is None else len(CBa), _dp(CBa), int(bool(correct)))
        if not self._h:
            raise ValueError("oracle: bad grid description")
        self.N = int(np.prod(self.n))
        self.dx = tuple(dx)
        self.dt = dt
        self.window = bool(window)

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_particles(self, x, u, Q, qm):
        """x: [np, ndim] cell-unit positions (x1 global), u: [np, 3] gamma*beta."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, self.ndim)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        assert x.shape[0] == u.shape[0]
        return lib().orc_add_particles(self._h, x.shape[0], _dp(x), _dp(u), float(Q), float(qm))

    def set_injection(self, ppc, Q, qm, uth, seed):
        p = (ctypes.c_int * 3)(*(list(ppc) + [1] * (3 - len(ppc))))
        lib().orc_set_injection(self._h, p, float(Q), float(qm), float(uth), ctypes.c_uint64(seed))

    def set_filter(self, npass, comp):
        """Smooth the current along x1 every step: npass binomial passes and a
        compensator of symbol 1 + comp sin^2(k dx1/2) (npass = 0: off)."""
        lib().orc_set_filter(self._h, int(npass), float(comp))

    def filter_j(self):
        lib().orc_filter_j(self._h)

    def step(self, nsteps=1):
        lib().orc_step(self._h, int(nsteps))

    def field_only(self, nsteps=1):
        lib().orc_field_only(self._h, int(nsteps))

    def field(self, name):
        out = np.empty(self.N, dtype=np.float64)
        lib().orc_get_field(self._h, FIELDS.index(name), _dp(out))
        return out.reshape(self.shape)

    def set_field(self, name, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        assert a.size == self.N
        lib().orc_set_field(self._h, FIELDS.index(name), _dp(a))

    @property
    def num_particles(self):
        return lib().orc_num_particles(self._h)

    @property
    def window_start(self):
        return lib().orc_window_start(self._h)

    @property
    def steps_done(self):
        return lib().orc_steps_done(self._h)

    def particles(self):
        npart = self.num_particles
        x = np.empty((npart, 3))
        u = np.empty((npart, 3))
        alive = np.empty(npart, dtype=np.int32)
        lib().orc_get_particles(self._h, _dp(x), _dp(u), alive.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return x[:, : self.ndim].copy(), u, alive.astype(bool)

    def rho(self):
        out = np.empty(self.N)
        lib().orc_rho(self._h, _dp(out))
        return out.reshape(self.shape)

    def div_e(self):
        out = np.empty(self.N)
        lib().orc_div_e(self._h, _dp(out))
        return out.reshape(self.shape)

    def energy(self):
        wf = ctypes.c_double()
        wk = ctypes.c_double()
        lib().orc_energy(self._h, ctypes.byref(wf), ctypes.byref(wk))
        return wf.value, wk.value

    def gather_at(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, self.ndim)
        out = np.empty((x.shape[0], 6))
        lib().orc_gather_at(self._h, x.shape[0], _dp(x), _dp(out))
        return out

    def deposit_one(self, Q, xo, xn, v3=0.0):
        a = np.ascontiguousarray(xo, dtype=np.float64)
        b = np.ascontiguousarray(xn, dtype=np.float64)
        lib().orc_deposit_one(self._h, float(Q), _dp(a), _dp(b), float(v3))

    def correct_j1(self):
        lib().orc_correct_j1(self._h)

    @property
    def correction_halfwidth(self):
        return lib().orc_correction_halfwidth(self._h)


def threads():
    """Threads the oracle's parallel loops use."""
    return int(lib().orc_max_threads())


def set_threads(n):
    """Use n threads in the parallel loops (results do not depend on n)."""
    lib().orc_set_threads(int(n))


def boris(qm, dt, EB, u):
    """One relativistic Boris push of u (gamma*beta) in fields EB = (E1,E2,E3,B1,B2,B3)."""
    EB = np.ascontiguousarray(EB, dtype=np.float64)
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    lib().orc_boris(float(qm), float(dt), _dp(EB), _dp(uu))
    return uu
