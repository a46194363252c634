"""ctypes binding of the C ABI in ``include/frelbm.h`` (argument marshalling
only: every step of the method runs in the HIP kernels of libfrelbm.so).

The functions keep the C names.  ``Lattice`` is a small convenience wrapper
that allocates the device buffer as a torch uint8 tensor and passes the torch
stream; it does no arithmetic of the method.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrelbm.so")

FRE_OK, FRE_EINVAL, FRE_ENOMEM, FRE_EDEVICE, FRE_ESTATE, FRE_ENUMERIC = 0, -1, -2, -3, -4, -5
FRE_D2Q9, FRE_D3Q19 = 0, 1
FRE_FP32, FRE_FP16 = 0, 1
FRE_PERIODIC, FRE_WALL = 0, 1
FRE_F_RHO, FRE_F_PHI, FRE_F_U, FRE_F_MU_RHO, FRE_F_MU_PHI, FRE_F_P = 1, 2, 4, 8, 16, 32
FRE_F_PSI, FRE_F_MU_PSI = 64, 128
FIELDS = (("rho", FRE_F_RHO), ("phi", FRE_F_PHI), ("u", FRE_F_U),
          ("mu_rho", FRE_F_MU_RHO), ("mu_phi", FRE_F_MU_PHI), ("P", FRE_F_P),
          ("psi", FRE_F_PSI), ("mu_psi", FRE_F_MU_PSI))


class FreError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"frelbm status {status}: {msg}")
        self.status = status


class fre_roller(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("radius", C.c_double), ("omega", C.c_double),
                ("axis", C.c_int32), ("reserved", C.c_int32)]


class fre_params(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("storage", C.c_int32), ("bc", C.c_int32 * 3),
        ("wall_u", ((C.c_double * 3) * 2) * 3),
        ("n_rollers", C.c_int32), ("fp16_rounding", C.c_int32),
        ("rollers", fre_roller * 4),
        ("A", C.c_double), ("kappa", C.c_double),
        ("kappa1", C.c_double), ("kappa2", C.c_double), ("alpha", C.c_double),
        ("use_paper_form", C.c_int32), ("ternary", C.c_int32),
        ("tau_f", C.c_double), ("tau_g", C.c_double), ("M", C.c_double),
        ("kappa3", C.c_double), ("M3", C.c_double), ("tau_h", C.c_double),
    ]


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("fre_footprint", C.c_int32, [C.POINTER(fre_params), C.POINTER(C.c_size_t)]),
    ("fre_lattice_init", C.c_int32, [C.POINTER(fre_params), C.c_void_p, C.c_size_t, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(C.c_void_p)]),
    ("fre_lattice_init3", C.c_int32, [C.POINTER(fre_params), C.c_void_p, C.c_size_t, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_void_p)]),
    ("fre_set_params", C.c_int32, [C.c_void_p, C.POINTER(fre_params)]),
    ("fre_consistent_init", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    ("fre_step", C.c_int32, [C.c_void_p, C.c_int64]),
    ("fre_read_moments", C.c_int32, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t]),
    ("fre_read_populations", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    ("fre_read_populations3", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    ("fre_reduce", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("fre_reduce_noalloc", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("fre_info", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    ("fre_state_bytes", C.c_int32, [C.c_void_p, C.POINTER(C.c_size_t)]),
    ("fre_save", C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("fre_load", C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("fre_profile_step", C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                                     C.POINTER(C.c_int32)]),
    ("fre_kernel_name", C.c_char_p, [C.c_int32]),
    ("fre_set_launch_shape", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("fre_get_launch_shape", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("fre_autotune", C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    ("fre_lattice_destroy", None, [C.c_void_p]),
    ("fre_batch_footprint", C.c_int32, [C.c_int32, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    ("fre_lattice_batch_needs", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("fre_batch_create", C.c_int32, [C.c_void_p, C.c_size_t, C.c_void_p, C.c_int32, C.c_int64, C.c_int64,
                                     C.POINTER(C.c_void_p)]),
    ("fre_batch_add", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    ("fre_batch_remove", C.c_int32, [C.c_void_p, C.c_int32]),
    ("fre_batch_step", C.c_int32, [C.c_void_p, C.c_int64]),
    ("fre_batch_info", C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("fre_batch_set_launch_shape", C.c_int32, [C.c_void_p, C.c_int32]),
    ("fre_batch_get_launch_shape", C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    ("fre_batch_autotune", C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("fre_batch_destroy", None, [C.c_void_p]),
    ("fre_last_error", C.c_char_p, []),
]


def lib():
    """Load libfrelbm.so; fails loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_01617_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != FRE_OK:
        raise FreError(status, lib().fre_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_params(kind, shape, *, storage=FRE_FP32, bc=(0, 0, 0), wall_u=None, rollers=(),
                A=None, kappa=None, kappa1=None, kappa2=None, alpha=None,
                tau_f=1.0, tau_g=1.0, M=0.1, ternary=None, stochastic_rounding=False) -> fre_params:
    """shape = (nx, ny, nz); rollers = [(center(3), omega, axis, radius)];
    give either (A, kappa) or (kappa1, kappa2, alpha).  A ternary lattice
    takes ternary=(kappa3, M3, tau_h).  stochastic_rounding (FP16 storage)
    sets fp16_rounding = 1."""
    p = fre_params()
    p.kind = kind
    p.nx, p.ny, p.nz = shape
    p.storage = storage
    for a in range(3):
        p.bc[a] = bc[a]
    if wall_u is not None:
        wu = np.asarray(wall_u, dtype=np.float64).reshape(3, 2, 3)
        for a in range(3):
            for s in range(2):
                for b in range(3):
                    p.wall_u[a][s][b] = wu[a, s, b]
    p.n_rollers = len(rollers)
    for k, r in enumerate(rollers):
        cen, om, ax = r[0], r[1], r[2]
        rad = r[3] if len(r) > 3 else 0.0
        for a in range(3):
            p.rollers[k].center[a] = cen[a]
        p.rollers[k].omega = om
        p.rollers[k].axis = ax
        p.rollers[k].radius = rad
    if kappa1 is not None:
        p.use_paper_form = 1
        p.kappa1, p.kappa2, p.alpha = kappa1, kappa2, alpha
    else:
        p.use_paper_form = 0
        p.A, p.kappa = A, kappa
    p.tau_f, p.tau_g, p.M = tau_f, tau_g, M
    if ternary is not None:
        p.ternary = 1
        p.kappa3, p.M3, p.tau_h = ternary
    p.fp16_rounding = 1 if stochastic_rounding else 0
    return p


def footprint(p: fre_params) -> int:
    n = C.c_size_t()
    _check(lib().fre_footprint(C.byref(p), C.byref(n)))
    return n.value


class Lattice:
    """A lattice in a torch-allocated device buffer, bound to a torch stream.
    Host fields are numpy arrays shaped (nz, ny, nx)."""

    def __init__(self, params: fre_params, phi0, rho0=None, u0=None, mask=None,
                 device="cuda:0", stream=None, psi0=None):
        """psi0 (ternary lattices, params.ternary = 1) is the third order
        parameter's initial field; the lattice is then made by
        fre_lattice_init3."""
        import torch  # device memory and streams only
        self.params = params
        self.ternary = bool(params.ternary)
        if self.ternary != (psi0 is not None):
            raise ValueError("psi0 is given exactly for ternary parameters")
        self.shape = (params.nz, params.ny, params.nx)
        self.N = params.nx * params.ny * params.nz
        self.q = 9 if params.kind == FRE_D2Q9 else 19
        nbytes = footprint(params)
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        self._base = self.buf.data_ptr() + off
        self._nbytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        phi0 = np.ascontiguousarray(np.asarray(phi0, np.float64).reshape(-1))
        rho0 = None if rho0 is None else np.ascontiguousarray(np.asarray(rho0, np.float64).reshape(-1))
        u0 = None if u0 is None else np.ascontiguousarray(np.asarray(u0, np.float64).reshape(-1))
        mask = None if mask is None else np.ascontiguousarray(np.asarray(mask, np.uint8).reshape(-1))
        h = C.c_void_p()
        rest = (None if rho0 is None else _ptr(rho0), None if u0 is None else _ptr(u0),
                None if mask is None else _ptr(mask), C.byref(h))
        if self.ternary:
            psi0 = np.ascontiguousarray(np.asarray(psi0, np.float64).reshape(-1))
            _check(lib().fre_lattice_init3(C.byref(params), C.c_void_p(self._base), nbytes,
                                           C.c_void_p(self.stream.cuda_stream), _ptr(phi0), _ptr(psi0), *rest))
        else:
            _check(lib().fre_lattice_init(C.byref(params), C.c_void_p(self._base), nbytes,
                                          C.c_void_p(self.stream.cuda_stream), _ptr(phi0), *rest))
        self._h = h

    def close(self):
        """Destroy the handle and release the device buffer once the
        lattice's stream has finished with it."""
        if getattr(self, "_h", None):
            lib().fre_lattice_destroy(self._h)
            self._h = None
            if getattr(self, "stream", None) is not None:
                self.stream.synchronize()
        self.buf = None

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if lib is not None:
            self.close()

    @property
    def handle(self):
        return self._h

    def consistent_init(self, phi0, u0=None, n: int = 100):
        """n (even) pre-iterations of f with u held at u0 and phi at phi0,
        then g reset to its equilibrium; only before the first step."""
        phi0 = np.ascontiguousarray(np.asarray(phi0, np.float64).reshape(-1))
        u0 = None if u0 is None else np.ascontiguousarray(np.asarray(u0, np.float64).reshape(-1))
        if phi0.size != self.N or (u0 is not None and u0.size != 3 * self.N):
            raise ValueError("phi0 needs N values and u0 3N")
        _check(lib().fre_consistent_init(self._h, _ptr(phi0), None if u0 is None else _ptr(u0), int(n)))
        return self

    def step(self, n=1):
        _check(lib().fre_step(self._h, int(n)))
        return self

    def set_params(self, params: fre_params):
        _check(lib().fre_set_params(self._h, C.byref(params)))
        self.params = params

    def read(self, fields=("rho", "phi", "u", "mu_rho", "mu_phi", "P")) -> dict:
        mask = 0
        for name, bit in FIELDS:
            if name in fields:
                mask |= bit
        n = sum((3 if name == "u" else 1) * self.N for name, bit in FIELDS if mask & bit)
        out = np.empty(n)
        _check(lib().fre_read_moments(self._h, mask, _ptr(out), n))
        res, o = {}, 0
        for name, bit in FIELDS:
            if mask & bit:
                k = 3 if name == "u" else 1
                a = out[o:o + k * self.N]
                res[name] = a.reshape((3,) + self.shape) if k == 3 else a.reshape(self.shape)
                o += k * self.N
        return res

    def populations(self):
        """(f, g), or (f, g, h) on a ternary lattice, each (q, nz, ny, nx)."""
        f = np.empty(self.q * self.N)
        g = np.empty(self.q * self.N)
        if self.ternary:
            h = np.empty(self.q * self.N)
            _check(lib().fre_read_populations3(self._h, _ptr(f), _ptr(g), _ptr(h), self.q * self.N))
            return tuple(a.reshape((self.q,) + self.shape) for a in (f, g, h))
        _check(lib().fre_read_populations(self._h, _ptr(f), _ptr(g), self.q * self.N))
        return f.reshape((self.q,) + self.shape), g.reshape((self.q,) + self.shape)

    def reduce(self) -> np.ndarray:
        out = np.zeros(8)
        _check(lib().fre_reduce(self._h, _ptr(out)))
        return out

    def reduce_noalloc(self) -> np.ndarray:
        """fre_reduce_noalloc: the same sums without any allocation by the
        library (calls on one GPU must not overlap)."""
        out = np.zeros(8)
        _check(lib().fre_reduce_noalloc(self._h, _ptr(out)))
        return out

    def info(self):
        t, s = C.c_int64(), C.c_int32()
        _check(lib().fre_info(self._h, C.byref(t), C.byref(s)))
        return t.value, s.value

    def profile(self, n: int) -> dict:
        """Mean per-step duration (ms) of each kernel of the step, from HIP
        events recorded around every launch on this lattice's stream."""
        ms = np.zeros(16)
        k = C.c_int32()
        _check(lib().fre_profile_step(self._h, int(n), _ptr(ms), 16, C.byref(k)))
        return {lib().fre_kernel_name(i).decode(): float(ms[i]) for i in range(k.value) if ms[i] >= 0.0}

    STAGES = ("k_moments", "k_potential", "k_collide")

    def launch_shape(self) -> dict:
        """{kernel: (rows, xcd)} for the three cell kernels."""
        cfg = np.zeros(6, np.int32)
        _check(lib().fre_get_launch_shape(self._h, _ptr(cfg)))
        return {k: (int(cfg[2 * i]), int(cfg[2 * i + 1])) for i, k in enumerate(self.STAGES)}

    def set_launch_shape(self, shape: dict):
        cfg = np.array([v for k in self.STAGES for v in shape[k]], np.int32)
        _check(lib().fre_set_launch_shape(self._h, _ptr(cfg)))

    def autotune(self, n: int = 10) -> dict:
        """Pick the fastest launch shape per cell kernel (state is restored);
        returns {kernel: (rows, xcd, ms)}."""
        cfg = np.zeros(6, np.int32)
        ms = np.zeros(3)
        _check(lib().fre_autotune(self._h, int(n), _ptr(cfg), _ptr(ms)))
        return {k: (int(cfg[2 * i]), int(cfg[2 * i + 1]), float(ms[i])) for i, k in enumerate(self.STAGES)}

    def save(self) -> bytes:
        n = C.c_size_t()
        _check(lib().fre_state_bytes(self._h, C.byref(n)))
        buf = np.empty(n.value, np.uint8)
        _check(lib().fre_save(self._h, _ptr(buf), n.value))
        return buf.tobytes()

    def load(self, blob: bytes):
        buf = np.frombuffer(blob, np.uint8).copy()
        _check(lib().fre_load(self._h, _ptr(buf), buf.size))


class Batch:
    """A batch of lattices advanced together (continuous batching): device
    tables in a torch-allocated buffer, steps on a torch stream."""

    def __init__(self, max_slots: int, max_work: int, max_fill: int, device="cuda:0", stream=None):
        import torch  # device memory and streams only
        n = C.c_size_t()
        _check(lib().fre_batch_footprint(max_slots, max_work, max_fill, C.byref(n)))
        self.buf = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr() + ((-self.buf.data_ptr()) % 256)
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        h = C.c_void_p()
        _check(lib().fre_batch_create(C.c_void_p(base), n.value, C.c_void_p(self.stream.cuda_stream),
                                      max_slots, max_work, max_fill, C.byref(h)))
        self._h = h
        self.members = {}

    @staticmethod
    def needs(lat: "Lattice"):
        w, f = C.c_int64(), C.c_int64()
        _check(lib().fre_lattice_batch_needs(lat.handle, C.byref(w), C.byref(f)))
        return w.value, f.value

    def add(self, lat: "Lattice") -> int:
        s = C.c_int32()
        _check(lib().fre_batch_add(self._h, lat.handle, C.byref(s)))
        self.members[s.value] = lat
        return s.value

    def remove(self, slot: int):
        _check(lib().fre_batch_remove(self._h, int(slot)))
        self.members.pop(slot, None)

    def step(self, n: int = 1):
        _check(lib().fre_batch_step(self._h, int(n)))
        return self

    def info(self):
        m, p = C.c_int32(), C.c_int32()
        _check(lib().fre_batch_info(self._h, C.byref(m), C.byref(p)))
        return m.value, p.value

    def launch_shape(self) -> int:
        """Persistent blocks per CU of the cell kernels."""
        b = C.c_int32()
        _check(lib().fre_batch_get_launch_shape(self._h, C.byref(b)))
        return b.value

    def set_launch_shape(self, blocks_per_cu: int):
        _check(lib().fre_batch_set_launch_shape(self._h, int(blocks_per_cu)))

    def autotune(self, n: int = 10):
        """Pick the fastest blocks per CU on the current members (their
        states are restored); returns (blocks_per_cu, ms/step)."""
        b = C.c_int32()
        ms = C.c_double()
        _check(lib().fre_batch_autotune(self._h, int(n), C.byref(b), C.byref(ms)))
        return b.value, ms.value

    def close(self):
        if getattr(self, "_h", None):
            lib().fre_batch_destroy(self._h)
            self._h = None
            self.members = {}

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if lib is not None:
            self.close()
