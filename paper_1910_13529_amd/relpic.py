"""Thin ctypes binding of librelpic.so (the C ABI in include/relpic.h).

Argument marshalling only: every step of the PIC cycle runs in the HIP
kernels of the library.  The functions keep the C names; `Sim` is a small
convenience wrapper.  PyTorch provides the device memory (through the
library's allocator callbacks) and the stream.  If the library is missing
this module raises: there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librelpic.so")

RELPIC_OK, RELPIC_EINVAL, RELPIC_EUNSTABLE, RELPIC_ERANGE, RELPIC_ENOMEM, RELPIC_EDEVICE, RELPIC_ESTATE = range(7)
RELPIC_FP32, RELPIC_FP64 = 0, 1
RELPIC_BC_PERIODIC, RELPIC_BC_WINDOW = 0, 1
FIELDS = ("E1", "E2", "E3", "B1", "B2", "B3", "J1", "J2", "J3")
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EUNSTABLE", 3: "ERANGE", 4: "ENOMEM", 5: "EDEVICE", 6: "ESTATE"}

EXPORTS = (
    "relpic_fit_coefficients", "relpic_create", "relpic_destroy", "relpic_add_species", "relpic_load_particles",
    "relpic_set_injection", "relpic_set_background_rho", "relpic_step", "relpic_sync", "relpic_read_field",
    "relpic_write_field", "relpic_field_device_ptr", "relpic_read_particles", "relpic_diagnostics",
    "relpic_get_step", "relpic_correction_halfwidth", "relpic_profile_enable", "relpic_profile_read",
    "relpic_sort_particles", "relpic_set_sort_interval", "relpic_set_fused_fields", "relpic_set_current_filter", "relpic_batch_create", "relpic_batch_destroy",
    "relpic_batch_run", "relpic_batch_step", "relpic_batch_sync", "relpic_batch_set_graph_steps",
    "relpic_batch_set_tiling", "relpic_batch_get_tiling", "relpic_batch_autotune", "relpic_batch_read_field",
    "relpic_adj_create", "relpic_adj_destroy", "relpic_adj_load_particles", "relpic_adj_forward",
    "relpic_adj_backward", "relpic_adj_sim", "relpic_kspace_e1", "relpic_kspace_field", "relpic_kspace_self_force", "relpic_gather_particles", "relpic_e1_residual",
    "relpic_kspace_e1_noalloc", "relpic_profile_read_species", "relpic_fit_operator", "relpic_init_beam_fields",
    "relpic_last_error",
)
KERNEL_CLASSES = ("push_deposit", "jcorr", "curl_e", "curl_b", "window", "add_j", "merge_boxes", "leap", "filter")


class RelpicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("bc1", ctypes.c_int), ("window_speed", ctypes.c_double)]


class Solver(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("C", ctypes.POINTER(ctypes.c_double)), ("MB", ctypes.c_int),
                ("CB", ctypes.POINTER(ctypes.c_double))]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Device(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("user", ctypes.c_void_p)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("window_start", ctypes.c_int64), ("n_alive", ctypes.c_int64),
                ("time", ctypes.c_double), ("w_field", ctypes.c_double), ("w_kin", ctypes.c_double),
                ("gauss_max", ctypes.c_double), ("rho_max", ctypes.c_double), ("charge", ctypes.c_double),
                ("error_word", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * len(KERNEL_CLASSES)), ("total_ms", ctypes.c_double * len(KERNEL_CLASSES))]


class BatchTune(ctypes.Structure):
    _fields_ = [("ms_uniform", ctypes.c_double * 3), ("ms_model", ctypes.c_double),
                ("ms_persistent", ctypes.c_double * 2), ("ms_chosen", ctypes.c_double), ("choice", ctypes.c_int),
                ("grid_workgroups", ctypes.c_int), ("runs_per_shape", ctypes.c_int * 3)]

    def as_dict(self):
        return {"ms_uniform": list(self.ms_uniform), "ms_model": self.ms_model,
                "ms_persistent": list(self.ms_persistent), "ms_chosen": self.ms_chosen, "choice": self.choice,
                "grid_workgroups": self.grid_workgroups, "runs_per_shape": list(self.runs_per_shape)}


class LossBox(ctypes.Structure):
    _fields_ = [("x1", ctypes.c_double), ("x2", ctypes.c_double), ("v1", ctypes.c_double),
                ("half1", ctypes.c_double), ("half2", ctypes.c_double)]


class KSpaceParams(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("C", ctypes.POINTER(ctypes.c_double)), ("kappa", ctypes.c_double),
                ("r", ctypes.c_double), ("beta", ctypes.c_double), ("shape_order", ctypes.c_int),
                ("tpow", ctypes.c_int), ("nu_max", ctypes.c_int), ("MB", ctypes.c_int),
                ("CB", ctypes.POINTER(ctypes.c_double))]


_lib = None


def load():
    """Load librelpic.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librelpic.so not built: run __graft_entry__.build() or python -m paper_1910_13529_amd.build")
    # PyTorch ships its own HIP runtime under the same soname as ROCm's.  Loaded
    # first, it is the one the library binds to, so the process has a single
    # runtime and torch's streams and allocations are the library's too;
    # loaded second, it would come up as a separate runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    for name in EXPORTS:
        getattr(L, name)  # every declared entry point must exist
    L.relpic_fit_coefficients.argtypes = [D, ctypes.c_int, ctypes.c_int, D, D, dp, dp]
    L.relpic_fit_operator.argtypes = [D, ctypes.c_int, ctypes.c_int, D, D, ctypes.c_int, dp, dp]
    L.relpic_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Solver), ctypes.c_int, ctypes.POINTER(Device),
                                ctypes.POINTER(P)]
    L.relpic_destroy.argtypes = [P]
    L.relpic_add_species.argtypes = [P, D, D, I64, ip]
    L.relpic_load_particles.argtypes = [P, ctypes.c_int, I64, ctypes.POINTER(ctypes.c_int32), dp, dp]
    L.relpic_set_injection.argtypes = [P, ctypes.c_int, ip, D, ctypes.c_uint64]
    L.relpic_set_background_rho.argtypes = [P, dp, I64]
    L.relpic_step.argtypes = [P, I64]
    L.relpic_sync.argtypes = [P]
    L.relpic_read_field.argtypes = [P, ctypes.c_int, dp, I64]
    L.relpic_write_field.argtypes = [P, ctypes.c_int, dp, I64]
    L.relpic_field_device_ptr.argtypes = [P, ctypes.c_int, ctypes.POINTER(P), ip]
    L.relpic_read_particles.argtypes = [P, ctypes.c_int, I64, ctypes.POINTER(ctypes.c_int32), dp, dp,
                                        ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.relpic_sort_particles.argtypes = [P]
    L.relpic_set_sort_interval.argtypes = [P, I64]
    L.relpic_set_fused_fields.argtypes = [P, ctypes.c_int, ip]
    L.relpic_set_current_filter.argtypes = [P, ctypes.c_int, D]
    L.relpic_diagnostics.argtypes = [P, ctypes.POINTER(Diag)]
    L.relpic_get_step.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.relpic_correction_halfwidth.argtypes = [P, ip]
    L.relpic_profile_enable.argtypes = [P, ctypes.c_int]
    L.relpic_profile_read.argtypes = [P, ctypes.POINTER(Profile)]
    L.relpic_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(Grid), ctypes.POINTER(Solver), ctypes.c_int,
                                      ctypes.POINTER(Device), ctypes.POINTER(P)]
    L.relpic_batch_destroy.argtypes = [P]
    L.relpic_batch_run.argtypes = [P, ctypes.c_int, ctypes.POINTER(P)]
    L.relpic_batch_step.argtypes = [P, I64]
    L.relpic_batch_sync.argtypes = [P]
    L.relpic_batch_set_graph_steps.argtypes = [P, ctypes.c_int]
    L.relpic_batch_set_tiling.argtypes = [P, ip, ctypes.c_int]
    L.relpic_batch_get_tiling.argtypes = [P, ip, ip]
    L.relpic_batch_autotune.argtypes = [P, ctypes.c_int, ctypes.POINTER(BatchTune)]
    L.relpic_batch_read_field.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, I64]
    L.relpic_adj_create.argtypes = [ctypes.POINTER(Grid), ctypes.c_int, dp, ctypes.c_int, ctypes.POINTER(Device), I64,
                                    ctypes.c_int, ctypes.POINTER(LossBox), ctypes.POINTER(P)]
    L.relpic_adj_destroy.argtypes = [P]
    L.relpic_adj_load_particles.argtypes = [P, D, I64, ctypes.POINTER(ctypes.c_int32), dp, dp]
    L.relpic_adj_forward.argtypes = [P, dp, dp]
    L.relpic_adj_backward.argtypes = [P, dp]
    L.relpic_adj_sim.argtypes = [P, ctypes.POINTER(P)]
    L.relpic_kspace_e1.argtypes = [ctypes.POINTER(KSpaceParams), ctypes.POINTER(Device), I64, dp, dp]
    L.relpic_kspace_field.argtypes = [ctypes.POINTER(KSpaceParams), ctypes.POINTER(Device), ctypes.c_int, D, I64, dp,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), dp]
    L.relpic_kspace_self_force.argtypes = [ctypes.POINTER(KSpaceParams), ctypes.POINTER(Device), ctypes.c_int, dp]
    L.relpic_profile_read_species.argtypes = [P, ctypes.c_int, ctypes.POINTER(I64), dp]
    L.relpic_init_beam_fields.argtypes = [P, D]
    L.relpic_kspace_e1_noalloc.argtypes = [ctypes.POINTER(KSpaceParams), ctypes.POINTER(Device), I64, dp, dp]
    L.relpic_gather_particles.argtypes = [P, ctypes.c_int, I64, I64, dp]
    L.relpic_e1_residual.argtypes = [P, ctypes.c_int, I64, ctypes.POINTER(KSpaceParams), I64,
                                     ctypes.POINTER(ctypes.c_int32), dp, dp]
    L.relpic_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "relpic_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(status):
    if status != RELPIC_OK:
        raise RelpicError(status, load().relpic_last_error().decode())
    return status


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- functions with the C names ------------------------------------------------------

def relpic_fit_coefficients(kappa, M, p=2, wk1=0.6, nsg=10.0):
    C = np.zeros(M)
    err = ctypes.c_double()
    check(load().relpic_fit_coefficients(kappa, M, p, wk1, nsg, _dp(C), ctypes.byref(err)))
    return C, err.value


RELPIC_FIT_TIME, RELPIC_FIT_E_WITH_YEE_B = 0, 1


def relpic_fit_operator(kappa, M, target=RELPIC_FIT_TIME, p=2, wk1=0.6, nsg=10.0):
    C = np.zeros(M)
    err = ctypes.c_double()
    check(load().relpic_fit_operator(kappa, M, p, wk1, nsg, int(target), _dp(C), ctypes.byref(err)))
    return C, err.value


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self._alloc = ALLOC_FN(self.alloc)
        self._free = FREE_FN(self.free)

    def alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda:%d" % self.device)
        except Exception:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def free(self, ptr, user):
        self.live.pop(ptr, None)


def _grid_struct(grid, g=None):
    g = Grid() if g is None else g
    g.ndim = grid["ndim"]
    for d in range(3):
        g.n[d] = int(grid["n"][d]) if d < g.ndim else 1
        g.dx[d] = float(grid["dx"][d]) if d < g.ndim else 1.0
    g.dt = float(grid["dt"])
    g.bc1 = RELPIC_BC_WINDOW if grid.get("window") else RELPIC_BC_PERIODIC
    g.window_speed = float(grid.get("window_speed", 1.0))
    return g


def _solver_struct(solver_C, s=None, CB=None):
    """fills a Solver (operator on E: solver_C; on B: CB, None = the same);
    returns it and the coefficient arrays it points to (keep them alive)"""
    s = Solver() if s is None else s
    Carr = None
    if solver_C is not None and len(solver_C) > 1:
        Carr = np.ascontiguousarray(solver_C, dtype=np.float64)
        s.M = len(Carr)
        s.C = _dp(Carr)
    else:
        s.M = 1
        s.C = None
    CBarr = None
    if CB is None:
        s.MB = 0
        s.CB = None
    else:
        CBarr = np.ascontiguousarray(CB, dtype=np.float64)
        s.MB = len(CBarr)
        s.CB = _dp(CBarr)
    return s, (Carr, CBarr)


def _device_struct(device, stream, allocator):
    dev = Device()
    dev.device = device
    dev.stream = stream
    if allocator is not None:
        dev.alloc = allocator._alloc
        dev.free = allocator._free
    return dev


def relpic_create(grid, solver_C=None, precision=RELPIC_FP64, device=0, stream=None, allocator=None, CB=None):
    L = load()
    g = _grid_struct(grid)
    s, Carr = _solver_struct(solver_C, CB=CB)
    dev = _device_struct(device, stream, allocator)
    h = ctypes.c_void_p()
    check(L.relpic_create(ctypes.byref(g), ctypes.byref(s), precision, ctypes.byref(dev), ctypes.byref(h)))
    return h


def relpic_destroy(h):
    return check(load().relpic_destroy(h))


def relpic_step(h, nsteps):
    return check(load().relpic_step(h, int(nsteps)))


def relpic_sync(h):
    return check(load().relpic_sync(h))


def _torch_binding(device):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("relpic needs a ROCm GPU (torch.cuda.is_available() is False)")
    torch.cuda.set_device(device)
    return TorchAllocator(device), torch.cuda.current_stream(device)


class SimOps:
    """The single-run calls on a handle (owned by a Sim or by a Batch)."""

    def _init_geometry(self, grid, precision):
        self.grid = dict(grid)
        self.ndim = grid["ndim"]
        self.n = tuple(int(v) for v in grid["n"][: self.ndim])
        self.N = int(np.prod(self.n))
        self.shape = tuple(reversed(self.n))
        self.prec = RELPIC_FP64 if precision in ("fp64", RELPIC_FP64) else RELPIC_FP32
        self.species = []

    def add_species(self, q_over_m, Q, capacity):
        sid = ctypes.c_int()
        check(load().relpic_add_species(self.h, float(q_over_m), float(Q), int(capacity), ctypes.byref(sid)))
        self.species.append(sid.value)
        return sid.value

    def load_particles(self, species, cell, offset, u):
        cell = np.ascontiguousarray(cell, dtype=np.int32).reshape(-1, self.ndim)
        offset = np.ascontiguousarray(offset, dtype=np.float64).reshape(-1, self.ndim)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        n = cell.shape[0]
        check(load().relpic_load_particles(self.h, species, n, cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           _dp(offset), _dp(u)))

    def set_injection(self, species, ppc, uth, seed):
        p = (ctypes.c_int * 3)(*(list(ppc) + [1] * (3 - len(ppc))))
        check(load().relpic_set_injection(self.h, species, p, float(uth), ctypes.c_uint64(seed)))

    def set_background_rho(self, rho):
        a = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        check(load().relpic_set_background_rho(self.h, _dp(a), a.size))

    def step(self, nsteps=1):
        relpic_step(self.h, nsteps)

    def sync(self):
        relpic_sync(self.h)

    def field(self, name):
        out = np.empty(self.N)
        check(load().relpic_read_field(self.h, FIELDS.index(name), _dp(out), self.N))
        return out.reshape(self.shape)

    def set_field(self, name, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        check(load().relpic_write_field(self.h, FIELDS.index(name), _dp(a), a.size))

    def field_device_ptr(self, name):
        p = ctypes.c_void_p()
        eb = ctypes.c_int()
        check(load().relpic_field_device_ptr(self.h, FIELDS.index(name), ctypes.byref(p), ctypes.byref(eb)))
        return p.value, eb.value

    def particles(self, species, cap, order_by_id=True):
        """(cell, offset, u, alive) of every slot; by default reordered by
        particle id (load order), so runs can be compared slot by slot."""
        cell = np.zeros((cap, self.ndim), dtype=np.int32)
        off = np.zeros((cap, self.ndim))
        u = np.zeros((cap, 3))
        alive = np.zeros(cap, dtype=np.uint8)
        ids = np.zeros(cap, dtype=np.int64)
        n = ctypes.c_int64()
        check(load().relpic_read_particles(self.h, species, cap, cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           _dp(off), _dp(u), alive.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                           ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(n)))
        k = n.value
        cell, off, u, alive, ids = cell[:k], off[:k], u[:k], alive[:k].astype(bool), ids[:k]
        if order_by_id:
            o = np.argsort(ids, kind="stable")
            cell, off, u, alive, ids = cell[o], off[o], u[o], alive[o], ids[o]
        self.last_ids = ids
        return cell, off, u, alive

    def sort_particles(self):
        check(load().relpic_sort_particles(self.h))

    def set_sort_interval(self, n):
        check(load().relpic_set_sort_interval(self.h, int(n)))

    def set_current_filter(self, npass, comp):
        """Current filter along x1: npass binomial passes and a compensator with c = comp (npass 0: off)."""
        check(load().relpic_set_current_filter(self.h, int(npass), float(comp)))

    def set_fused_fields(self, enable):
        """Fused E and B update (3D grids that qualify); returns whether it is active."""
        a = ctypes.c_int(0)
        check(load().relpic_set_fused_fields(self.h, 1 if enable else 0, ctypes.byref(a)))
        return bool(a.value)

    def diagnostics(self):
        d = Diag()
        check(load().relpic_diagnostics(self.h, ctypes.byref(d)))
        return d.as_dict()

    def get_step(self):
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        check(load().relpic_get_step(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def profile_enable(self, on=True):
        check(load().relpic_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        p = Profile()
        check(load().relpic_profile_read(self.h, ctypes.byref(p)))
        return {k: (int(p.launches[i]), float(p.total_ms[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def init_beam_fields(self, beta):
        """Self-consistent fields of the loaded charges moving along x1 at beta (relpic_init_beam_fields)."""
        check(load().relpic_init_beam_fields(self.h, float(beta)))

    def gather_particles(self, species, first=0, count=None):
        """E1..B3 (FP64, [count, 6]) at the particles of slots first .. first + count - 1."""
        if count is None:
            count = self.num_slots(species) - first
        out = np.zeros((int(count), 6))
        check(load().relpic_gather_particles(self.h, species, int(first), int(count), _dp(out)))
        return out

    def num_slots(self, species):
        n = ctypes.c_int64()
        st = load().relpic_read_particles(self.h, species, 0, None, None, None, None, None, ctypes.byref(n))
        if st not in (RELPIC_OK, RELPIC_ERANGE):
            check(st)
        return n.value

    def e1_residual(self, species, slot, i1_rel, C=None, kappa=None, r=None, beta=1.0, shape_order=2, tpow=1,
                    nu_max=3):
        """(simulated, k-space) E1 at E1 points i1_rel on the particle's row around the particle in
        `slot`: E1 dx1 / Q in 2D, E1 dx1^2 / Q in 3D (relpic_e1_residual)."""
        g = self.grid
        if C is None:
            C, CB = getattr(self, "C", None), getattr(self, "CB", None)
        else:
            CB = None
        kappa = g["dx"][0] / g["dt"] if kappa is None else kappa
        r = g["dx"][1] / g["dx"][0] if r is None else r
        q, keep = _kspace_struct(C, kappa, r, beta, shape_order, tpow, nu_max, CB)
        rel = np.ascontiguousarray(i1_rel, dtype=np.int32)
        sim = np.zeros(rel.size)
        th = np.zeros(rel.size)
        check(load().relpic_e1_residual(self.h, species, int(slot), ctypes.byref(q), rel.size,
                                        rel.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(sim), _dp(th)))
        return sim, th

    def profile_read_species(self, species):
        """(launches, total ms) of one species' push+deposit since profiling was enabled."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        check(load().relpic_profile_read_species(self.h, species, ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    @property
    def correction_halfwidth(self):
        v = ctypes.c_int()
        check(load().relpic_correction_halfwidth(self.h, ctypes.byref(v)))
        return v.value


class Sim(SimOps):
    """One simulation on one GPU.  grid: dict(ndim, n, dx, dt, window, window_speed)."""

    def __init__(self, grid, C=None, precision="fp64", device=0, use_torch=True, CB=None):
        """C: the axial operator on E (and on B unless CB gives that one)."""
        self._init_geometry(grid, precision)
        self.C = None if C is None or len(C) <= 1 else np.array(C, dtype=np.float64)
        self.CB = None if CB is None else np.array(CB, dtype=np.float64)
        self.allocator = None
        stream = None
        if use_torch:
            self.allocator, self.torch_stream = _torch_binding(device)
            stream = self.torch_stream.cuda_stream
        self.h = relpic_create(grid, C, self.prec, device, stream, self.allocator, CB=CB)

    def close(self):
        if getattr(self, "h", None):
            load().relpic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchRun(SimOps):
    """A run of a Batch (the handle belongs to the batch)."""

    def __init__(self, batch, index, grid):
        self._init_geometry(grid, batch.prec)
        self.batch = batch
        self.index = index
        h = ctypes.c_void_p()
        check(load().relpic_batch_run(batch.h, index, ctypes.byref(h)))
        self.h = h


class Batch:
    """Many independent 2D periodic runs advanced together (relpic_batch_*).
    grids: list of grid dicts; Cs: list of coefficient arrays (None = Yee)."""

    def __init__(self, grids, Cs=None, precision="fp32", device=0):
        n = len(grids)
        self.prec = RELPIC_FP64 if precision in ("fp64", RELPIC_FP64) else RELPIC_FP32
        self.allocator, self.torch_stream = _torch_binding(device)
        garr = (Grid * n)()
        sarr = (Solver * n)()
        keep = []
        for r, g in enumerate(grids):
            _grid_struct(g, garr[r])
            _, Carr = _solver_struct(None if Cs is None else Cs[r], sarr[r])
            keep.append(Carr)
        dev = _device_struct(device, self.torch_stream.cuda_stream, self.allocator)
        h = ctypes.c_void_p()
        check(load().relpic_batch_create(n, garr, sarr, self.prec, ctypes.byref(dev), ctypes.byref(h)))
        self.h = h
        self.runs = [BatchRun(self, r, g) for r, g in enumerate(grids)]

    def __len__(self):
        return len(self.runs)

    def step(self, nsteps=1):
        check(load().relpic_batch_step(self.h, int(nsteps)))

    def sync(self):
        check(load().relpic_batch_sync(self.h))

    def set_graph_steps(self, steps):
        check(load().relpic_batch_set_graph_steps(self.h, int(steps)))

    def set_tiling(self, shapes=None, grid_workgroups=0):
        arr = None
        if shapes is not None:
            a = np.ascontiguousarray(shapes, dtype=np.int32)
            arr = a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        check(load().relpic_batch_set_tiling(self.h, arr, int(grid_workgroups)))

    def tiling(self):
        a = np.zeros(len(self.runs), dtype=np.int32)
        g = ctypes.c_int()
        check(load().relpic_batch_get_tiling(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                             ctypes.byref(g)))
        return a, g.value

    def autotune(self, reps=10):
        t = BatchTune()
        check(load().relpic_batch_autotune(self.h, int(reps), ctypes.byref(t)))
        return t.as_dict()

    def field(self, run, name):
        r = self.runs[run]
        out = np.empty(r.N)
        check(load().relpic_batch_read_field(self.h, run, FIELDS.index(name), _dp(out), r.N))
        return out.reshape(r.shape)

    def close(self):
        if getattr(self, "h", None):
            for r in self.runs:
                r.h = None
            load().relpic_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Adjoint:
    """Loss of the fields around a ballistic bunch and its gradient with
    respect to the axial coefficients (relpic_adj_*).  grid: 2D periodic grid
    dict; C0: initial coefficients (length M); box: dict(x1, x2, v1, half1,
    half2) of the excluded region."""

    def __init__(self, grid, C0, nsteps, box, checkpoint_every=20, precision="fp32", device=0):
        self.prec = RELPIC_FP64 if precision in ("fp64", RELPIC_FP64) else RELPIC_FP32
        self.allocator, self.torch_stream = _torch_binding(device)
        self.M = len(C0)
        g = _grid_struct(grid)
        C = np.ascontiguousarray(C0, dtype=np.float64)
        lb = LossBox(*(float(box[k]) for k in ("x1", "x2", "v1", "half1", "half2")))
        dev = _device_struct(device, self.torch_stream.cuda_stream, self.allocator)
        h = ctypes.c_void_p()
        check(load().relpic_adj_create(ctypes.byref(g), self.M, _dp(C), self.prec, ctypes.byref(dev), int(nsteps),
                                       int(checkpoint_every), ctypes.byref(lb), ctypes.byref(h)))
        self.h = h
        self.grid = grid

    def load_particles(self, Q, cell, offset, u):
        cell = np.ascontiguousarray(cell, dtype=np.int32).reshape(-1, 2)
        offset = np.ascontiguousarray(offset, dtype=np.float64).reshape(-1, 2)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        check(load().relpic_adj_load_particles(self.h, float(Q), cell.shape[0],
                                               cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(offset),
                                               _dp(u)))

    def forward(self, C):
        C = np.ascontiguousarray(C, dtype=np.float64)
        assert C.size == self.M
        out = np.zeros(1)
        check(load().relpic_adj_forward(self.h, _dp(C), _dp(out)))
        return float(out[0])

    def backward(self):
        g = np.zeros(self.M)
        check(load().relpic_adj_backward(self.h, _dp(g)))
        return g

    def sim(self):
        """The simulation the adjoint runs on (fields of the last forward pass)."""
        h = ctypes.c_void_p()
        check(load().relpic_adj_sim(self.h, ctypes.byref(h)))
        v = SimOps()
        v._init_geometry(self.grid, self.prec)
        v.h = h
        return v

    def close(self):
        if getattr(self, "h", None):
            load().relpic_adj_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def adjoint_loss(adj, C):
    """torch.autograd.Function: loss(C) with dL/dC from the adjoint pass.
    C: a 1-D float64 CPU tensor of length adj.M (requires_grad for training)."""
    import torch

    class _AdjointLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, c):
            loss = adj.forward(c.detach().cpu().numpy().astype(np.float64))
            return torch.tensor(loss, dtype=c.dtype)

        @staticmethod
        def backward(ctx, grad_out):
            g = torch.from_numpy(adj.backward()).to(grad_out.dtype)
            return grad_out * g

    return _AdjointLoss.apply(C)


def _kspace_struct(C, kappa, r, beta, order, tpow, nu_max, CB=None):
    q = KSpaceParams()
    Carr = np.ascontiguousarray([1.0] if C is None else C, dtype=np.float64)
    q.M = Carr.size
    q.C = _dp(Carr)
    q.kappa, q.r, q.beta = float(kappa), float(r), float(beta)
    q.shape_order, q.tpow, q.nu_max = int(order), int(tpow), int(nu_max)
    CBarr = None
    if CB is None:
        q.MB, q.CB = 0, None
    else:
        CBarr = np.ascontiguousarray(CB, dtype=np.float64)
        q.MB, q.CB = CBarr.size, _dp(CBarr)
    return q, (Carr, CBarr)


def kspace_e1(i1_rel, C=None, kappa=4.0, r=1.0, beta=1.0, order=2, tpow=0, nu_max=1, device=0, CB=None):
    """On-axis E1 dx1 / q of a streaming charge at E1 points i1_rel cells
    ahead of it (relpic_kspace_e1; FP64 quadrature on the GPU)."""
    q, keep = _kspace_struct(C, kappa, r, beta, order, tpow, nu_max, CB)
    x = np.ascontiguousarray(np.atleast_1d(i1_rel), dtype=np.float64)
    out = np.zeros(x.size)
    dev = _device_struct(device, None, None)
    check(load().relpic_kspace_e1(ctypes.byref(q), ctypes.byref(dev), x.size, _dp(x), _dp(out)))
    return out


def kspace_field(i1_rel, i2=0, i3=None, C=None, kappa=4.0, r=1.0, r3=None, beta=1.0, order=2, tpow=0, nu_max=1,
                 device=0, CB=None):
    """E1 at E1 points (i1_rel + 1/2, i2[, i3]) of a 2D grid (i3 and r3 None:
    E1 dx1 / q) or a 3D grid (E1 dx1^2 / q, r3 = dx3/dx1), by
    relpic_kspace_field."""
    q, keep = _kspace_struct(C, kappa, r, beta, order, tpow, nu_max, CB)
    x = np.ascontiguousarray(np.atleast_1d(i1_rel), dtype=np.float64)
    j2 = np.ascontiguousarray(np.broadcast_to(np.asarray(i2, dtype=np.int32), x.shape))
    ndim = 2 if i3 is None else 3
    j3 = np.ascontiguousarray(np.broadcast_to(np.asarray(0 if i3 is None else i3, dtype=np.int32), x.shape))
    out = np.zeros(x.size)
    dev = _device_struct(device, None, None)
    ip = ctypes.POINTER(ctypes.c_int32)
    check(load().relpic_kspace_field(ctypes.byref(q), ctypes.byref(dev), ndim, float(1.0 if r3 is None else r3), x.size,
                                     _dp(x), j2.ctypes.data_as(ip), j3.ctypes.data_as(ip), _dp(out)))
    return out


def kspace_e1_noalloc(i1_rel, C=None, kappa=4.0, r=1.0, beta=1.0, order=2, tpow=0, nu_max=1, device=0):
    """relpic_kspace_e1 without device allocation (library-held scratch)."""
    q, keep = _kspace_struct(C, kappa, r, beta, order, tpow, nu_max)
    x = np.ascontiguousarray(np.atleast_1d(i1_rel), dtype=np.float64)
    out = np.zeros(x.size)
    dev = _device_struct(device, None, None)
    check(load().relpic_kspace_e1_noalloc(ctypes.byref(q), ctypes.byref(dev), x.size, _dp(x), _dp(out)))
    return out


def kspace_self_force(C=None, kappa=4.0, r=1.0, beta=1.0, order=2, tpow=0, nu_max=1, gather_order=None, device=0):
    """Self-force F1 dx1 / q^2 (relpic_kspace_self_force)."""
    q, keep = _kspace_struct(C, kappa, r, beta, order, tpow, nu_max)
    out = np.zeros(1)
    dev = _device_struct(device, None, None)
    check(load().relpic_kspace_self_force(ctypes.byref(q), ctypes.byref(dev),
                                          int(order if gather_order is None else gather_order), _dp(out)))
    return float(out[0])
