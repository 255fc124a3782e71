"""ctypes binding of ``liborc.so`` (the FP64 CPU oracle, ``orc.c``).

TEST INFRASTRUCTURE ONLY.  Argument marshalling; no arithmetic of the method.
Arrays use the lattice layout of the C code: a scalar field is a float64 array
of shape (nz, ny, nx) (x fastest); a vector field is (3, nz, ny, nx); the
populations are (7, nz, ny, nx) and (15, nz, ny, nx) ((19, ...) for COUPLED_Q19).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ORC_LIB_PATH") or os.path.join(_HERE, "liborc.so")

PERIODIC, WALL = 0, 1
COUPLED, CHE_ONLY, COUPLED_Q19 = 0, 1, 2
STENCIL_Q15, STENCIL_Q7 = 0, 1
FORCING_EQ32, FORCING_EQ28 = 0, 1
FIELDS = {"phi": 0, "rho": 1, "mu": 2, "ux": 3, "uy": 4, "uz": 5, "p": 6}
VEL_ZERO, VEL_FIELD, VEL_ZALESAK, VEL_DEFORM = 0, 1, 2, 3
E_NONFINITE = 5


SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, sanitize: bool = False, path: str = None) -> str:
    """Compile orc.c into liborc.so (gcc, FP64, no FMA contraction, OpenMP).
    sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build (host
    code, for checking the oracle itself; load it with the sanitizer runtimes
    preloaded, see sanitizer_env)."""
    out = path or LIB_PATH
    opt = SANITIZE_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-Wall", "-o", out, os.path.join(_HERE, "orc.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


def sanitizer_env(lib_path: str) -> dict:
    """Environment for a Python process that loads a sanitizer build of the
    oracle: the runtimes preloaded (Python itself is not instrumented), leak
    checks off (the interpreter keeps its allocations), any finding fatal."""
    rt = [subprocess.run(["gcc", "-print-file-name=" + n], capture_output=True, text=True,
                         check=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    env = dict(os.environ)
    env.update({"LD_PRELOAD": ":".join(rt), "ORC_LIB_PATH": lib_path,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    return env


class OrcParams(C.Structure):
    _fields_ = [("sigma", C.c_double), ("width", C.c_double), ("rho_l", C.c_double),
                ("rho_g", C.c_double), ("mobility", C.c_double), ("A", C.c_double),
                ("s_f", C.c_double * 7), ("nu", C.c_double), ("lambda_g", C.c_double * 15),
                ("gravity", C.c_double * 3), ("rho_ref", C.c_double),
                ("stencil", C.c_int), ("forcing", C.c_int), ("lambda_override", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library not built: {LIB_PATH}")
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, ip, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_params.argtypes = [C.c_void_p, C.POINTER(OrcParams)]
        L.orc_init.argtypes = [C.c_void_p, dp, dp]
        L.orc_set_velocity.argtypes = [C.c_void_p, C.c_int, dp, C.c_double, C.c_double]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_step_count.restype = C.c_long
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_read.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_totals.argtypes = [C.c_void_p, dp]
        L.orc_lattice19.argtypes = [ip, dp, dp]
        L.orc_geq19.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_T.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_front.argtypes = [C.c_void_p, dp]
        L.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_last_error.restype = C.c_char_p
        L.orc_last_error.argtypes = [C.c_void_p]
        L.orc_matrices.argtypes = [dp, dp]
        L.orc_lattices.argtypes = [C.c_double, ip, dp, ip, dp]
        L.orc_derived.argtypes = [C.POINTER(OrcParams), dp]
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_geq.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_meq_f.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_mR.argtypes = [dp, dp]
        L.orc_meq_g.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_mT.argtypes = [dp, dp, dp, dp]
        L.orc_grad_lap.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.argtypes = []
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's OpenMP loops (timing only)."""
    if lib().orc_set_threads(int(n)) != 0:
        raise ValueError(f"thread count {n}")


def threads():
    return int(lib().orc_get_threads())


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def to_params(p) -> OrcParams:
    """Copy a parameter record (any object with the ModelParams attributes)."""
    o = OrcParams()
    o.sigma, o.width, o.rho_l, o.rho_g = p.sigma, p.width, p.rho_l, p.rho_g
    o.mobility, o.A, o.nu, o.rho_ref = p.mobility, p.A, p.nu, p.rho_ref
    for i in range(7):
        o.s_f[i] = p.s_f[i]
    for i in range(15):
        o.lambda_g[i] = p.lambda_g[i]
    for a in range(3):
        o.gravity[a] = p.gravity[a]
    o.stencil = int(getattr(p, "stencil", 0))
    o.forcing = int(getattr(p, "forcing", 0))
    o.lambda_override = int(getattr(p, "lambda_override", 0))
    return o


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """One lattice of the oracle.  shape = (nx, ny, nz); bc = per-axis PERIODIC/WALL."""

    def __init__(self, shape, bc=(PERIODIC, PERIODIC, PERIODIC), mode=COUPLED, params=None):
        L = lib()
        self.nx, self.ny, self.nz = (int(v) for v in shape)
        bca = (C.c_int * 3)(*bc)
        self._h = L.orc_create(self.nx, self.ny, self.nz, bca, int(mode))
        if not self._h:
            raise OracleError(1, "orc_create failed")
        self.mode = mode
        if params is not None:
            self.set_params(params)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().orc_destroy(h)
            except TypeError:  # interpreter shutdown: the module's globals are gone
                pass
            self._h = None

    def _chk(self, rc):
        if rc != 0:
            raise OracleError(rc, lib().orc_last_error(self._h).decode())

    @property
    def grid(self):
        return (self.nz, self.ny, self.nx)

    def set_params(self, p):
        self._p = to_params(p)
        self._chk(lib().orc_set_params(self._h, C.byref(self._p)))

    def set_velocity(self, kind, field=None, U=0.0, T=1.0):
        fa = None if field is None else _f64(field)
        self._chk(lib().orc_set_velocity(self._h, int(kind), _dp(fa), float(U), float(T)))

    def init(self, phi0, u0=None):
        phi0 = _f64(phi0)
        u0 = None if u0 is None else _f64(u0)
        self._chk(lib().orc_init(self._h, _dp(phi0), _dp(u0)))

    def step(self, n=1):
        self._chk(lib().orc_step(self._h, int(n)))

    def try_step(self, n=1):
        """Step and return (code, message) instead of raising."""
        rc = lib().orc_step(self._h, int(n))
        return rc, lib().orc_last_error(self._h).decode()

    @property
    def step_count(self):
        return int(lib().orc_step_count(self._h))

    def read(self, field):
        out = np.empty(self.grid, dtype=np.float64)
        self._chk(lib().orc_read(self._h, FIELDS[field], _dp(out)))
        return out

    def read_all(self):
        return {k: self.read(k) for k in FIELDS}

    def totals(self):
        out = np.empty(7, dtype=np.float64)
        self._chk(lib().orc_totals(self._h, _dp(out)))
        return out

    def front(self):
        """(lowest, highest) z of a zero crossing of phi along z; (-1, -1) if none."""
        out = np.empty(2, dtype=np.float64)
        self._chk(lib().orc_front(self._h, _dp(out)))
        return out

    def get_state(self):
        f = np.empty((7,) + self.grid)
        g = np.empty((19 if self.mode == COUPLED_Q19 else 15,) + self.grid)
        pu = np.empty((3,) + self.grid)
        self._chk(lib().orc_get_state(self._h, _dp(f), _dp(g), _dp(pu)))
        return f, g, pu

    def set_state(self, f=None, g=None, phiu=None):
        f = None if f is None else _f64(f)
        g = None if g is None else _f64(g)
        phiu = None if phiu is None else _f64(phiu)
        self._chk(lib().orc_set_state(self._h, _dp(f), _dp(g), _dp(phiu)))

    def grad_lap(self, chi):
        chi = _f64(chi)
        gr = np.empty((3,) + self.grid)
        lp = np.empty(self.grid)
        self._chk(lib().orc_grad_lap(self._h, _dp(chi), _dp(gr), _dp(lp)))
        return gr, lp


# ---- node-level pieces ----

def matrices():
    M = np.empty((7, 7))
    G = np.empty((15, 15))
    lib().orc_matrices(_dp(M), _dp(G))
    return M, G


def lattices(A=0.25):
    c7 = np.empty((7, 3), dtype=np.int32)
    c15 = np.empty((15, 3), dtype=np.int32)
    w7 = np.empty(7)
    w15 = np.empty(15)
    ip = C.POINTER(C.c_int)
    lib().orc_lattices(float(A), c7.ctypes.data_as(ip), _dp(w7), c15.ctypes.data_as(ip), _dp(w15))
    return c7, w7, c15, w15


def derived(p):
    """(beta, k, tau_f, eta, tau_g, lambda_visc)."""
    out = np.empty(6)
    pp = to_params(p)
    lib().orc_derived(C.byref(pp), _dp(out))
    return out


def feq(A, eta, phi, mu, u):
    out = np.empty(7)
    lib().orc_feq(float(A), float(eta), float(phi), float(mu), _dp(_f64(u)), _dp(out))
    return out


def geq(p, rho, u):
    out = np.empty(15)
    lib().orc_geq(float(p), float(rho), _dp(_f64(u)), _dp(out))
    return out


def meq_f(A, eta, phi, mu, u):
    out = np.empty(7)
    lib().orc_meq_f(float(A), float(eta), float(phi), float(mu), _dp(_f64(u)), _dp(out))
    return out


def mR(dphiu):
    out = np.empty(7)
    lib().orc_mR(_dp(_f64(dphiu)), _dp(out))
    return out


def meq_g(p, rho, u):
    out = np.empty(15)
    lib().orc_meq_g(float(p), float(rho), _dp(_f64(u)), _dp(out))
    return out


def mT(u, grad_rho, F):
    out = np.empty(15)
    lib().orc_mT(_dp(_f64(u)), _dp(_f64(grad_rho)), _dp(_f64(F)), _dp(out))
    return out


def lattice19():
    """(c19 (19, 3), w19 (19,), Gamma_19 (19, 19)) of the D3Q19 variant."""
    c = np.empty((19, 3), dtype=np.int32)
    w = np.empty(19)
    G = np.empty((19, 19))
    lib().orc_lattice19(c.ctypes.data_as(C.POINTER(C.c_int)), _dp(w), _dp(G))
    return c, w, G


def geq19(p, rho, u):
    out = np.empty(19)
    lib().orc_geq19(float(p), float(rho), _dp(_f64(u)), _dp(out))
    return out


def T(q, u, grad_rho, F):
    """Eq. 28 on D3Q15 (q = 15) or D3Q19 (q = 19)."""
    out = np.empty(q)
    lib().orc_T(int(q), _dp(_f64(u)), _dp(_f64(grad_rho)), _dp(_f64(F)), _dp(out))
    return out
