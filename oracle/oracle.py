"""ctypes front end of the FP64 CPU oracle (``frelbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the independent reference the GPU path is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; it shares no code with the GPU library and never
imports it.

The oracle follows Sec. 2.2-2.3 and Algorithm 1 of Simonis et al. (arXiv
2212.01617); the readings taken where the paper is silent are listed at the
top of ``frelbm_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "frelbm_oracle.c")
_LIB = os.path.join(_HERE, "libfrelbm_oracle.so")


def compile_source(src: str, out: str) -> str:
    """gcc build of an oracle source file (FP64, no FMA contraction, OpenMP)."""
    tmp = out + ".tmp"
    subprocess.check_call([
        "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        "-Wno-unused-parameter", src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle (when the library is missing or older than the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


class Params(C.Structure):
    """Mirror of ``or_params`` in frelbm_oracle.c."""
    _fields_ = [
        ("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 3),
        ("wall_u", ((C.c_double * 3) * 2) * 3),
        ("n_rollers", C.c_int32),
        ("roller_center", (C.c_double * 3) * 4),
        ("roller_omega", C.c_double * 4),
        ("roller_axis", C.c_int32 * 4),
        ("kappa1", C.c_double), ("kappa2", C.c_double), ("alpha", C.c_double),
        ("tau_f", C.c_double), ("tau_g", C.c_double), ("M", C.c_double),
    ]


_lib = None


def lib():
    """The compiled oracle.  FRELBM_ORACLE_LIB names another build of the same
    source to load instead (the mutation tests plant mistakes in copies)."""
    global _lib
    if _lib is None:
        path = os.environ.get("FRELBM_ORACLE_LIB") or build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.or_tables.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
        L.or_feq.argtypes = [C.c_int, C.c_double, dp, dp]
        L.or_guo.argtypes = [C.c_int, C.c_double, dp, dp, dp]
        L.or_geq.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp]
        L.or_mu.argtypes = [C.c_double] * 7 + [dp]
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(Params), C.c_void_p, dp, dp, dp]
        L.or_create_geometry.restype = C.c_void_p
        L.or_create_geometry.argtypes = [C.POINTER(Params), C.c_void_p]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_step.argtypes = [C.c_void_p, C.c_long]
        L.or_consistent_init.argtypes = [C.c_void_p, dp, C.c_void_p, C.c_long]
        L.or_consistent_init.restype = C.c_int
        L.or_time.argtypes = [C.c_void_p]
        L.or_time.restype = C.c_long
        L.or_observe.argtypes = [C.c_void_p, dp]
        L.or_get_populations.argtypes = [C.c_void_p, dp, dp]
        L.or_set_populations.argtypes = [C.c_void_p, dp, dp]
        L.or_stencils.argtypes = [C.c_void_p, dp, dp, dp]
        L.or3_mu.argtypes = [C.c_double] * 10 + [dp]
        L.or3_psi_bulk.argtypes = [C.c_double] * 6
        L.or3_psi_bulk.restype = C.c_double
        L.or3_create.restype = C.c_void_p
        L.or3_create.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double, C.c_void_p, dp, dp, dp, dp]
        L.or3_step.argtypes = [C.c_void_p, C.c_long]
        L.or3_observe.argtypes = [C.c_void_p, dp]
        L.or3_get_populations.argtypes = [C.c_void_p, dp, dp, dp]
        L.or3_set_populations.argtypes = [C.c_void_p, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# --------------------------------------------------------------------------
# per-node formulas (for the moment-identity pins)
# --------------------------------------------------------------------------
def tables(kind: int):
    q = C.c_int()
    c = (C.c_int * (19 * 3))()
    w = np.zeros(19)
    if lib().or_tables(kind, C.byref(q), c, _dp(w)) != 0:
        raise ValueError(kind)
    n = q.value
    return np.array(c[: 3 * n], dtype=np.int64).reshape(n, 3), w[:n].copy()


def feq(kind, rho, u):
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().or_feq(kind, rho, _dp(uu), _dp(out))
    return out[: 9 if kind == 0 else 19]


def guo(kind, tau, u, F):
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    FF = np.ascontiguousarray(F, dtype=np.float64)
    lib().or_guo(kind, tau, _dp(uu), _dp(FF), _dp(out))
    return out[: 9 if kind == 0 else 19]


def geq(kind, phi, mu_phi, Gamma, u):
    out = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().or_geq(kind, phi, mu_phi, Gamma, _dp(uu), _dp(out))
    return out[: 9 if kind == 0 else 19]


def mu(kappa1, kappa2, alpha, rho, phi, lap_rho, lap_phi):
    out = np.zeros(2)
    lib().or_mu(kappa1, kappa2, alpha, rho, phi, lap_rho, lap_phi, _dp(out))
    return out[0], out[1]


def paper_form(A: float, kappa: float):
    """(A, kappa) of the symmetric binary free energy -> (kappa1, kappa2, alpha)
    of eq. (functional): with kappa1 = kappa2 = 4A the bulk term is
    A/4 (phi^2-1)^2 and the gradient term alpha^2 kappa1/4 |grad phi|^2 equals
    kappa/2 |grad phi|^2, so alpha = sqrt(kappa / (2A))."""
    return 4.0 * A, 4.0 * A, float(np.sqrt(kappa / (2.0 * A)))


# --------------------------------------------------------------------------
# lattice
# --------------------------------------------------------------------------
OBS_FIELDS = ("rho", "phi", "ux", "uy", "uz", "mu_rho", "mu_phi", "P", "solid")


def make_params(kind, shape, *, bc=(0, 0, 0), wall_u=None, rollers=(),
                kappa1=None, kappa2=None, alpha=None, A=None, kappa=None,
                tau_f=1.0, tau_g=1.0, M=0.1) -> Params:
    """shape = (nx, ny, nz); rollers = [(center(3), omega, axis)]."""
    p = Params()
    p.kind = kind
    p.nx, p.ny, p.nz = shape
    for a in range(3):
        p.bc[a] = bc[a]
    if wall_u is not None:
        wu = np.asarray(wall_u, dtype=np.float64).reshape(3, 2, 3)
        for a in range(3):
            for s in range(2):
                for b in range(3):
                    p.wall_u[a][s][b] = wu[a, s, b]
    p.n_rollers = len(rollers)
    for k, (cen, om, ax) in enumerate(rollers):
        for a in range(3):
            p.roller_center[k][a] = cen[a]
        p.roller_omega[k] = om
        p.roller_axis[k] = ax
    if A is not None:
        kappa1, kappa2, alpha = paper_form(A, kappa)
    p.kappa1, p.kappa2, p.alpha = kappa1, kappa2, alpha
    p.tau_f, p.tau_g, p.M = tau_f, tau_g, M
    return p


class Lattice:
    """One oracle lattice.  Fields are numpy arrays shaped (nz, ny, nx)."""

    def __init__(self, params: Params, phi0, rho0=None, u0=None, mask=None):
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        self.N = params.nx * params.ny * params.nz
        self.q = 9 if params.kind == 0 else 19
        phi0 = np.ascontiguousarray(np.asarray(phi0, dtype=np.float64).reshape(-1))
        rho0 = None if rho0 is None else np.ascontiguousarray(np.asarray(rho0, np.float64).reshape(-1))
        u0 = None if u0 is None else np.ascontiguousarray(np.asarray(u0, np.float64).reshape(3, -1))
        self._mask = None if mask is None else np.ascontiguousarray(np.asarray(mask, np.uint8).reshape(-1))
        self._keep = (phi0, rho0, u0)
        self._h = lib().or_create(C.byref(params),
                                  None if self._mask is None else self._mask.ctypes.data,
                                  _dp(phi0),
                                  None if rho0 is None else _dp(rho0),
                                  None if u0 is None else _dp(u0))
        if not self._h:
            raise ValueError("oracle rejected the lattice parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:  # module globals are gone at interpreter exit
            lib().or_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return lib().or_time(self._h)

    def step(self, n: int = 1):
        lib().or_step(self._h, int(n))
        return self

    def consistent_init(self, phi0, u0=None, n: int = 100):
        """n pre-iterations of f with u held at u0 and phi at phi0, then g
        reset to its equilibrium (Sec. 2.3, after Mei et al. 2006)."""
        phi0 = np.ascontiguousarray(np.asarray(phi0, dtype=np.float64).reshape(-1))
        u0 = None if u0 is None else np.ascontiguousarray(np.asarray(u0, np.float64).reshape(-1))
        r = lib().or_consistent_init(self._h, _dp(phi0), None if u0 is None else u0.ctypes.data, int(n))
        if r != 0:
            raise ValueError("consistent initialisation is only possible before the first step")
        return self

    def observe(self) -> dict:
        out = np.zeros(9 * self.N)
        lib().or_observe(self._h, _dp(out))
        out = out.reshape(9, *self.shape)
        return {k: out[i] for i, k in enumerate(OBS_FIELDS)}

    def populations(self):
        f = np.zeros(self.q * self.N)
        g = np.zeros(self.q * self.N)
        lib().or_get_populations(self._h, _dp(f), _dp(g))
        return f.reshape(self.q, *self.shape), g.reshape(self.q, *self.shape)

    def set_populations(self, f, g):
        f = np.ascontiguousarray(np.asarray(f, np.float64).reshape(-1))
        g = np.ascontiguousarray(np.asarray(g, np.float64).reshape(-1))
        lib().or_set_populations(self._h, _dp(f), _dp(g))

    def stencils(self, X):
        X = np.ascontiguousarray(np.asarray(X, np.float64).reshape(-1))
        lap = np.zeros(self.N)
        grad = np.zeros(3 * self.N)
        lib().or_stencils(self._h, _dp(X), _dp(lap), _dp(grad))
        return lap.reshape(self.shape), grad.reshape(3, *self.shape)


# --------------------------------------------------------------------------
# ternary extension (Sec. 2.2, Remark after the mobility relation)
# --------------------------------------------------------------------------
def mu3(kappa1, kappa2, kappa3, alpha, rho, phi, psi, lap_rho, lap_phi, lap_psi):
    """(mu_rho, mu_phi, mu_psi) of the ternary free energy at a node."""
    out = np.zeros(3)
    lib().or3_mu(kappa1, kappa2, kappa3, alpha, rho, phi, psi, lap_rho, lap_phi, lap_psi, _dp(out))
    return tuple(out)


def psi_bulk3(kappa1, kappa2, kappa3, rho, phi, psi):
    """Bulk free-energy density of the ternary functional."""
    return lib().or3_psi_bulk(kappa1, kappa2, kappa3, rho, phi, psi)


OBS3_FIELDS = ("rho", "phi", "psi", "ux", "uy", "uz", "mu_rho", "mu_phi", "mu_psi", "P", "solid")


class Lattice3:
    """A ternary oracle lattice: the binary parameters (phi's mobility M,
    tau_g) plus kappa3 and psi's mobility M3 and relaxation time tau_h.
    Fields are numpy arrays shaped (nz, ny, nx)."""

    def __init__(self, params: Params, kappa3, M3, tau_h, phi0, psi0, rho0=None, u0=None, mask=None):
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        self.N = params.nx * params.ny * params.nz
        self.q = 9 if params.kind == 0 else 19
        phi0 = np.ascontiguousarray(np.asarray(phi0, dtype=np.float64).reshape(-1))
        psi0 = np.ascontiguousarray(np.asarray(psi0, dtype=np.float64).reshape(-1))
        rho0 = None if rho0 is None else np.ascontiguousarray(np.asarray(rho0, np.float64).reshape(-1))
        u0 = None if u0 is None else np.ascontiguousarray(np.asarray(u0, np.float64).reshape(3, -1))
        self._mask = None if mask is None else np.ascontiguousarray(np.asarray(mask, np.uint8).reshape(-1))
        self._keep = (phi0, psi0, rho0, u0)
        self._h = lib().or3_create(C.byref(params), float(kappa3), float(M3), float(tau_h),
                                   None if self._mask is None else self._mask.ctypes.data,
                                   _dp(phi0), _dp(psi0),
                                   None if rho0 is None else _dp(rho0),
                                   None if u0 is None else _dp(u0))
        if not self._h:
            raise ValueError("oracle rejected the lattice parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and lib is not None:
            lib().or_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return lib().or_time(self._h)

    def step(self, n: int = 1):
        lib().or3_step(self._h, int(n))
        return self

    def observe(self) -> dict:
        out = np.zeros(11 * self.N)
        lib().or3_observe(self._h, _dp(out))
        out = out.reshape(11, *self.shape)
        return {k: out[i] for i, k in enumerate(OBS3_FIELDS)}

    def populations(self):
        f = np.zeros(self.q * self.N)
        g = np.zeros(self.q * self.N)
        h = np.zeros(self.q * self.N)
        lib().or3_get_populations(self._h, _dp(f), _dp(g), _dp(h))
        return tuple(a.reshape(self.q, *self.shape) for a in (f, g, h))

    def set_populations(self, f, g, h):
        f, g, h = (np.ascontiguousarray(np.asarray(a, np.float64).reshape(-1)) for a in (f, g, h))
        lib().or3_set_populations(self._h, _dp(f), _dp(g), _dp(h))
