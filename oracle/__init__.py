"""CPU oracle of the IDP Q1 Euler scheme -- TEST INFRASTRUCTURE ONLY.

Thin ctypes binding of ``idp_oracle.c`` (plain scalar FP64 C, one function
per building block of the paper's method).  Only ``tests/``, the package
smoke check and the benchmark's CPU-baseline leg may import this module; the
HIP library never does, and the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "idp_oracle.c")
# IDP_ORACLE_SANITIZE=1 builds and loads a copy instrumented with the
# address and undefined-behaviour sanitizers (the host process must then
# preload the sanitizer runtimes; see the design notes for the command)
_SANITIZE = os.environ.get("IDP_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libidp_oracle_san.so" if _SANITIZE else "libidp_oracle.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
              "-fno-omit-frame-pointer", "-g"]

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-Wall", *(_SAN_FLAGS if _SANITIZE else []),
             "-o", tmp, _SRC, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


_libs = {}


def load_library(path: str = _LIB):
    """The oracle library at ``path`` with its ctypes signatures (cached per
    path; the default is the oracle built from ``idp_oracle.c``)."""
    L = _libs.get(path)
    if L is not None:
        return L
    if path == _LIB and not os.path.exists(_LIB):
        build()
    L = C.CDLL(path)
    L.ora_create.restype = C.c_void_p
    L.ora_create.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int,
                             C.c_int, C.c_double, C.c_int, C.c_int64, _dp,
                             C.c_int64, _i64p, _u8p, C.POINTER(C.c_int)]
    L.ora_destroy.argtypes = [C.c_void_p]
    L.ora_max_dt.restype = C.c_double
    L.ora_max_dt.argtypes = [C.c_void_p, _dp]
    L.ora_euler_stage.restype = C.c_int
    L.ora_euler_stage.argtypes = [C.c_void_p, _dp, C.c_double, _dp]
    L.ora_step.restype = C.c_int
    L.ora_step.argtypes = [C.c_void_p, _dp, C.c_double, _dp]
    L.ora_n.restype = C.c_int64
    L.ora_n.argtypes = [C.c_void_p]
    L.ora_nnz.restype = C.c_int64
    L.ora_nnz.argtypes = [C.c_void_p]
    L.ora_volume.restype = C.c_double
    L.ora_volume.argtypes = [C.c_void_p]
    L.ora_set_literal_alg3.argtypes = [C.c_void_p, C.c_int]
    L.ora_set_limiter_mode.argtypes = [C.c_void_p, C.c_int]
    L.ora_set_threads.restype = C.c_int
    L.ora_set_threads.argtypes = [C.c_int]
    L.ora_array.restype = C.c_void_p
    L.ora_array.argtypes = [C.c_void_p, C.c_int]
    for name in ("ora_pressure", "ora_speed_of_sound",
                 "ora_specific_entropy", "ora_harten_entropy"):
        f = getattr(L, name)
        f.restype = C.c_double
        f.argtypes = [_dp, C.c_int, C.c_double]
    L.ora_harten_entropy_derivative.argtypes = [_dp, C.c_int, C.c_double, _dp]
    L.ora_pow.restype = C.c_double
    L.ora_pow.argtypes = [C.c_double, C.c_double]
    L.ora_lambda_max.restype = C.c_double
    L.ora_lambda_max.argtypes = [_dp, _dp, _dp, C.c_int, C.c_double, _dp]
    L.ora_limiter.restype = C.c_double
    L.ora_limiter.argtypes = [_dp, _dp, _dp, C.c_int, C.c_double, C.c_int,
                              C.c_double, C.c_int]
    _libs[path] = L
    return L


def lib():
    return load_library(_LIB)


def build_variant(source: str, path: str) -> str:
    """Compile the oracle from the C text ``source`` into ``path`` with the
    oracle's own flags (tests plant mistakes this way to show that a pin
    catches them)."""
    src = path + ".c"
    with open(src, "w") as f:
        f.write(source)
    subprocess.run(
        ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
         "-fPIC", "-shared", "-o", path, src, "-lm"], check=True)
    return path


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return int(lib().ora_set_threads(int(n)))


# ------------------------------------------------------------ pointwise

def pressure(U, gamma=1.4):
    U, p = _d(U)
    return lib().ora_pressure(p, U.shape[0] - 2, gamma)


def speed_of_sound(U, gamma=1.4):
    U, p = _d(U)
    return lib().ora_speed_of_sound(p, U.shape[0] - 2, gamma)


def specific_entropy(U, gamma=1.4):
    U, p = _d(U)
    return lib().ora_specific_entropy(p, U.shape[0] - 2, gamma)


def harten_entropy(U, gamma=1.4):
    U, p = _d(U)
    return lib().ora_harten_entropy(p, U.shape[0] - 2, gamma)


def harten_entropy_derivative(U, gamma=1.4):
    U, p = _d(U)
    out = np.zeros(U.shape[0])
    lib().ora_harten_entropy_derivative(p, U.shape[0] - 2, gamma,
                                        out.ctypes.data_as(_dp))
    return out


def pow_(x, y):
    """The oracle's fixed-method x^y (x > 0)."""
    return lib().ora_pow(float(x), float(y))


def lambda_max(n, Ui, Uj, gamma=1.4):
    """(lambda~_max, p*) of the paper's guaranteed wave-speed bound."""
    n, pn = _d(n)
    Ui, pi = _d(Ui)
    Uj, pj = _d(Uj)
    ps = C.c_double(0.0)
    lam = lib().ora_lambda_max(pn, pi, pj, n.shape[0], gamma, C.byref(ps))
    return lam, ps.value


def limiter(U, P, bounds, gamma=1.4, newton_max=2, tol=1e-10, literal=False):
    U, pu = _d(U)
    P, pp = _d(P)
    b, pb = _d(bounds)
    return lib().ora_limiter(pu, pp, pb, U.shape[0] - 2, gamma,
                             int(newton_max), tol, int(bool(literal)))


# ------------------------------------------------------------- solver

class Oracle:
    """Whole-mesh oracle: graph, matrices, forward-Euler stage, SSP-RK3."""

    def __init__(self, mesh=None, *, dim=None, coords=None, cells=None,
                 dirichlet=None, gamma=1.4, cfl=0.5, passes=2, newton_max=2,
                 newton_tol=1e-10, relax=False, library=None):
        self._L = load_library(library) if library else lib()
        if mesh is not None:
            dim, coords, cells = mesh.dim, mesh.coords, mesh.cells
            if dirichlet is None:
                dirichlet = mesh.boundary
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        n = coords.shape[0]
        if dirichlet is None:
            dirichlet = np.zeros(n, dtype=np.uint8)
        dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        err = C.c_int(0)
        self.dim, self.nc, self.gamma, self.cfl = dim, dim + 2, gamma, cfl
        self._h = self._L.ora_create(
            dim, gamma, cfl, passes, newton_max, newton_tol, int(relax), n,
            coords.ctypes.data_as(_dp), cells.shape[0],
            cells.ctypes.data_as(_i64p), dirichlet.ctypes.data_as(_u8p),
            C.byref(err))
        if not self._h:
            raise ValueError(f"oracle create failed: {err.value}")
        self.n = int(self._L.ora_n(self._h))
        self.nnz = int(self._L.ora_nnz(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.ora_destroy(h)
            self._h = None

    def set_literal_alg3(self, on: bool):
        self._L.ora_set_literal_alg3(self._h, int(bool(on)))

    LIMITER_MODES = {"paper": 0, "high": 1, "low": 2}

    def set_limiter_mode(self, mode: str):
        """'paper': Alg. 2 candidates; 'high': every l_ij = 1 (the unlimited
        high-order update); 'low': every l_ij = 0 (the low-order update)."""
        self._L.ora_set_limiter_mode(self._h, self.LIMITER_MODES[mode])

    @property
    def volume(self):
        return self._L.ora_volume(self._h)

    def _arr(self, what, dtype, count, shape=None):
        ptr = self._L.ora_array(self._h, what)
        ctype = {np.int64: C.c_int64, np.float64: C.c_double}[dtype]
        a = np.ctypeslib.as_array(C.cast(ptr, C.POINTER(ctype)), shape=(count,))
        a = a.copy()
        return a.reshape(shape) if shape is not None else a

    # matrices
    def row_ptr(self): return self._arr(0, np.int64, self.n + 1)
    def col(self): return self._arr(1, np.int64, self.nnz)
    def tpos(self): return self._arr(2, np.int64, self.nnz)
    def m_ij(self): return self._arr(3, np.float64, self.nnz)
    def c_ij(self): return self._arr(4, np.float64, self.nnz * self.dim, (self.nnz, self.dim))
    def m_i(self): return self._arr(5, np.float64, self.n)
    def lam(self): return self._arr(6, np.float64, self.n)
    # intermediates of the last stage
    def d_ij(self): return self._arr(7, np.float64, self.nnz)
    def alpha(self): return self._arr(8, np.float64, self.n)
    def R(self): return self._arr(9, np.float64, self.n * self.nc, (self.n, self.nc))
    def U_low(self): return self._arr(10, np.float64, self.n * self.nc, (self.n, self.nc))
    def bounds(self): return self._arr(11, np.float64, self.n * 3, (self.n, 3))
    def P(self): return self._arr(12, np.float64, self.nnz * self.nc, (self.nnz, self.nc))
    def l1(self): return self._arr(13, np.float64, self.nnz)
    def l2(self): return self._arr(14, np.float64, self.nnz)
    def U_pass1(self): return self._arr(15, np.float64, self.n * self.nc, (self.n, self.nc))
    def tau_i(self): return self._arr(16, np.float64, self.n)

    def max_dt(self, U):
        U, p = _d(U)
        return self._L.ora_max_dt(self._h, p)

    def euler_stage(self, U, tau):
        """Forward-Euler update E(U) with limiting; returns (Unew, warn)."""
        U, p = _d(U)
        out = np.empty_like(U)
        w = self._L.ora_euler_stage(self._h, p, tau, out.ctypes.data_as(_dp))
        return out, int(w)

    def step(self, U, dt=0.0):
        """One SSP-RK3 step; returns (Unew, dt_used, status)."""
        U = np.array(U, dtype=np.float64, copy=True, order="C")
        used = C.c_double(0.0)
        st = self._L.ora_step(self._h, U.ctypes.data_as(_dp), float(dt),
                            C.byref(used))
        return U, used.value, int(st)
