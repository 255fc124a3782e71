"""Thin ctypes binding of libmplb (include/mplb.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libmplb.so.  Device memory is a torch tensor (the lattice's arena) and work is
enqueued on torch's current stream.  There is no CPU fallback: without the
built library or a GPU the calls raise.

Host arrays use the lattice layout: a scalar field is float64 of shape
(nz, ny, nx) (x fastest); a vector field is (3, nz, ny, nx).
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmplb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mplb.h")

# constants of include/mplb.h
MPLB_OK, MPLB_E_INVAL, MPLB_E_NOMEM, MPLB_E_DEVICE, MPLB_E_STATE, MPLB_E_NONFINITE = 0, 1, 2, 3, 4, 5
MPLB_PERIODIC, MPLB_WALL = 0, 1
MPLB_F64, MPLB_F32, MPLB_F32_F16, MPLB_F32_BF16 = 0, 1, 2, 3
MPLB_COUPLED, MPLB_CHE_ONLY, MPLB_COUPLED_Q19 = 0, 1, 2
MPLB_PHI, MPLB_RHO, MPLB_MU, MPLB_UX, MPLB_UY, MPLB_UZ, MPLB_P = range(7)
MPLB_VEL_ZERO, MPLB_VEL_FIELD, MPLB_VEL_ZALESAK, MPLB_VEL_DEFORM = 0, 1, 2, 3

FIELDS = {"phi": MPLB_PHI, "rho": MPLB_RHO, "mu": MPLB_MU, "ux": MPLB_UX, "uy": MPLB_UY, "uz": MPLB_UZ,
          "p": MPLB_P}
PRECISIONS = {"f64": MPLB_F64, "f32": MPLB_F32, "f16": MPLB_F32_F16, "bf16": MPLB_F32_BF16}
VELOCITIES = {"zero": MPLB_VEL_ZERO, "field": MPLB_VEL_FIELD, "zalesak": MPLB_VEL_ZALESAK,
              "deformation": MPLB_VEL_DEFORM}


class mplb_params(C.Structure):
    _fields_ = [("sigma", C.c_double), ("width", C.c_double), ("rho_l", C.c_double),
                ("rho_g", C.c_double), ("mobility", C.c_double), ("A", C.c_double),
                ("s_f", C.c_double * 7), ("nu", C.c_double), ("lambda_g", C.c_double * 15),
                ("gravity", C.c_double * 3), ("rho_ref", C.c_double),
                ("stencil", C.c_int), ("forcing", C.c_int), ("lambda_override", C.c_int)]


class MplbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mplb error {code} ({_strerror(code)}): {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmplb.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmplb.so is not built ({LIB_PATH}); run paper_1507_07294_amd/build.py")
        # torch ships its own HIP runtime under the same soname as the system
        # one; loading torch first makes libmplb bind to that copy, so that
        # torch's memory and streams and the library share one runtime
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp, ip, sz = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_size_t
        sig = {
            "mplb_required_bytes": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(sz)]),
            "mplb_create": (C.c_int, [C.c_int, C.c_int, C.c_int, ip, C.c_int, C.c_int, vp, sz, C.POINTER(vp)]),
            "mplb_set_stream": (C.c_int, [vp, vp]),
            "mplb_set_params": (C.c_int, [vp, C.POINTER(mplb_params)]),
            "mplb_set_velocity": (C.c_int, [vp, C.c_int, dp, C.c_double, C.c_double]),
            "mplb_init": (C.c_int, [vp, dp, dp]),
            "mplb_step": (C.c_int, [vp, C.c_int]),
            "mplb_set_check_interval": (C.c_int, [vp, C.c_int]),
            "mplb_step_count": (C.c_long, [vp]),
            "mplb_read": (C.c_int, [vp, C.c_int, dp]),
            "mplb_read_diagonal": (C.c_int, [vp, C.c_int, dp]),
            "mplb_totals": (C.c_int, [vp, dp]),
            "mplb_front": (C.c_int, [vp, dp]),
            "mplb_step_many": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int]),
            "mplb_step_many_noalloc": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int]),
            "mplb_check_finite": (C.c_int, [vp]),
            "mplb_set_step_many_graphs": (C.c_int, [C.c_int]),
            "mplb_checkpoint_bytes": (C.c_int, [vp, C.POINTER(sz)]),
            "mplb_checkpoint": (C.c_int, [vp, vp, sz]),
            "mplb_restore": (C.c_int, [vp, vp, sz]),
            "mplb_poke": (C.c_int, [vp, C.c_int, C.c_int, C.c_long, C.c_double]),
            "mplb_force_tile_rows": (C.c_int, [vp, C.c_int]),
            "mplb_launch_shape": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, ip]),
            "mplb_poison": (C.c_int, [vp]),
            "mplb_time_stages": (C.c_int, [vp, C.c_int, dp]),
            "mplb_copy_probe": (C.c_int, [vp, vp, sz, C.c_int, vp]),
            "mplb_destroy": (None, [vp]),
            "mplb_last_error": (C.c_char_p, [vp]),
            "mplb_strerror": (C.c_char_p, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    """Entry points declared in include/mplb.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mplb_[a-z_]+)\s*\(", txt)))


def _strerror(code):
    try:
        return lib().mplb_strerror(int(code)).decode()
    except Exception:  # library not loadable: still report the code
        return "?"


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def to_params(p) -> mplb_params:
    """Copy a parameter record (any object with the ModelParams attributes)."""
    o = mplb_params()
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


SHAPE_KINDS = ("coupled, 64 x 8 tiles", "coupled, 64 x 16 tiles", "CHE-only, one node per thread",
               "CHE-only, two nodes per thread")


def mplb_launch_shape(nx, ny, nz, precision, mode, rows=0):
    """The kernel and work split mplb_step uses for such a lattice (host
    computation): kind (index into SHAPE_KINDS), tile width and height,
    planes per segment, segments and blocks."""
    out = (C.c_int * 6)()
    rc = lib().mplb_launch_shape(nx, ny, nz, precision, mode, rows, out)
    if rc:
        raise MplbError(rc, "mplb_launch_shape")
    return {"kind": out[0], "tile": (out[1], out[2]), "lz": out[3], "segments": out[4], "blocks": out[5]}


def mplb_required_bytes(nx, ny, nz, precision, mode):
    out = C.c_size_t(0)
    rc = lib().mplb_required_bytes(nx, ny, nz, precision, mode, C.byref(out))
    if rc:
        raise MplbError(rc, "mplb_required_bytes")
    return int(out.value)


class Lattice:
    """One lattice of libmplb; the handle's C calls keep their names as methods
    (mplb_step -> step, mplb_read -> read, ...)."""

    def __init__(self, shape, bc=(0, 0, 0), precision="f64", mode=MPLB_COUPLED, params=None, arena=None,
                 device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libmplb needs a ROCm GPU; torch.cuda is not available")
        L = lib()
        self.nx, self.ny, self.nz = (int(v) for v in shape)
        self.N = self.nx * self.ny * self.nz
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.mode = int(mode)
        self.bc = tuple(int(b) for b in bc)
        nbytes = mplb_required_bytes(self.nx, self.ny, self.nz, self.precision, self.mode)
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        # device memory comes from torch; the library borrows it until destroy()
        self.arena = arena if arena is not None else torch.empty(nbytes, dtype=torch.uint8, device=dev)
        if self.arena.numel() < nbytes:
            raise ValueError("arena too small")
        h = C.c_void_p()
        bca = (C.c_int * 3)(*self.bc)
        rc = L.mplb_create(self.nx, self.ny, self.nz, bca, self.precision, self.mode,
                           C.c_void_p(self.arena.data_ptr()), C.c_size_t(self.arena.numel()), C.byref(h))
        if rc:
            raise MplbError(rc, "mplb_create")
        self._h = h
        self.set_stream(torch.cuda.current_stream(dev).cuda_stream)
        if params is not None:
            self.set_params(params)

    @property
    def handle(self):
        return self._h

    def _chk(self, rc):
        if rc:
            raise MplbError(rc, lib().mplb_last_error(self._h).decode())

    @property
    def grid(self):
        return (self.nz, self.ny, self.nx)

    def set_stream(self, stream_ptr):
        self._chk(lib().mplb_set_stream(self._h, C.c_void_p(int(stream_ptr))))

    def set_params(self, p):
        self._params = to_params(p)
        self._chk(lib().mplb_set_params(self._h, C.byref(self._params)))

    def set_velocity(self, kind, field=None, U=0.0, T=1.0):
        kind = VELOCITIES[kind] if isinstance(kind, str) else int(kind)
        fa = None if field is None else _f64(field, 3 * self.N)
        self._chk(lib().mplb_set_velocity(self._h, kind, _dp(fa), float(U), float(T)))

    def init(self, phi0, u0=None):
        phi0 = _f64(phi0, self.N)
        u0 = None if u0 is None else _f64(u0, 3 * self.N)
        self._chk(lib().mplb_init(self._h, _dp(phi0), _dp(u0)))

    def set_check_interval(self, k):
        self._chk(lib().mplb_set_check_interval(self._h, int(k)))

    def step(self, n=1):
        self._chk(lib().mplb_step(self._h, int(n)))

    def check_finite(self):
        """MPLB_OK, or MPLB_E_NONFINITE if a population of this lattice became
        non-finite since init (synchronises)."""
        rc = lib().mplb_check_finite(self._h)
        if rc not in (MPLB_OK, MPLB_E_NONFINITE):
            self._chk(rc)
        return rc

    def last_error(self):
        return lib().mplb_last_error(self._h).decode()

    def try_step(self, n=1):
        rc = lib().mplb_step(self._h, int(n))
        return rc, lib().mplb_last_error(self._h).decode()

    @property
    def step_count(self):
        return int(lib().mplb_step_count(self._h))

    def read(self, field):
        out = np.empty(self.grid, dtype=np.float64)
        self._chk(lib().mplb_read(self._h, FIELDS[field] if isinstance(field, str) else int(field), _dp(out)))
        return out

    def read_diagonal(self, field):
        """The field on the vertical plane x = y (nx = ny), shape (nz, nx):
        [z, i] is the value at node (i, i, z); gathered on the device."""
        nz, _, nx = self.grid
        out = np.empty((nz, nx), dtype=np.float64)
        self._chk(lib().mplb_read_diagonal(self._h, FIELDS[field] if isinstance(field, str) else int(field),
                                           _dp(out)))
        return out

    def read_all(self):
        return {k: self.read(k) for k in FIELDS}

    def totals(self):
        out = np.empty(7, dtype=np.float64)
        self._chk(lib().mplb_totals(self._h, _dp(out)))
        return out

    def front(self):
        """(spike tip, bubble front): lowest and highest z of a zero crossing of
        phi along z at the current level; (-1, -1) if there is none."""
        out = np.empty(2, dtype=np.float64)
        self._chk(lib().mplb_front(self._h, _dp(out)))
        return out

    def try_totals(self):
        out = np.empty(7, dtype=np.float64)
        rc = lib().mplb_totals(self._h, _dp(out))
        return rc, out

    def checkpoint(self):
        n = C.c_size_t(0)
        self._chk(lib().mplb_checkpoint_bytes(self._h, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._chk(lib().mplb_checkpoint(self._h, buf.ctypes.data_as(C.c_void_p), n))
        return buf

    def restore(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._chk(lib().mplb_restore(self._h, buf.ctypes.data_as(C.c_void_p), C.c_size_t(buf.size)))

    def time_stages(self, n):
        """Advance n steps and return the summed event-timed milliseconds of (phi pass, mu pass,
        step kernel, whole step); one kernel does the whole step, so the first two are 0."""
        out = np.zeros(4, dtype=np.float64)
        self._chk(lib().mplb_time_stages(self._h, int(n), _dp(out)))
        return out

    def poke(self, set_, i, node, value):
        self._chk(lib().mplb_poke(self._h, int(set_), int(i), int(node), float(value)))

    def poison(self):
        """Test hook: NaN-fill what the next step writes and the padding it must
        not read, and have later steps NaN-fill their LDS first."""
        self._chk(lib().mplb_poison(self._h))

    def force_tile_rows(self, rows):
        """Test hook: tile height of the coupled step (0 automatic, 8 or 16)."""
        self._chk(lib().mplb_force_tile_rows(self._h, int(rows)))

    def destroy(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().mplb_destroy(h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


MPLB_NOALLOC_MAX_LATTICES = 512


def _many(fn, lattices, nsteps):
    arr = (C.c_void_p * len(lattices))(*[lt.handle.value for lt in lattices])
    rc = fn(arr, len(lattices), int(nsteps))
    if rc:
        if rc == MPLB_E_NONFINITE:
            bad = [i for i, lt in enumerate(lattices) if lt.check_finite() == MPLB_E_NONFINITE]
            raise NonFiniteError(bad, [lattices[i].last_error() for i in bad])
        raise MplbError(rc, lib().mplb_last_error(lattices[0].handle).decode() if lattices else "")


class NonFiniteError(MplbError):
    """mplb_step_many found non-finite populations; `failed` lists the
    positions of the failed lattices in the batch, `messages` their errors."""

    def __init__(self, failed, messages):
        super().__init__(MPLB_E_NONFINITE, "; ".join(messages))
        self.failed = list(failed)
        self.messages = list(messages)


def mplb_step_many(lattices, nsteps):
    """Advance several lattices together (batched launches).  Raises
    NonFiniteError naming the failed lattices when a non-finite check fails."""
    _many(lib().mplb_step_many, lattices, nsteps)


def mplb_step_many_noalloc(lattices, nsteps):
    """mplb_step_many with no device or host allocation (static batch table of
    MPLB_NOALLOC_MAX_LATTICES lattices per device, launches one by one)."""
    _many(lib().mplb_step_many_noalloc, lattices, nsteps)


def mplb_set_step_many_graphs(enable):
    """Replay batched steps as a graph (True, the default) or launch them one by one."""
    rc = lib().mplb_set_step_many_graphs(1 if enable else 0)
    if rc:
        raise MplbError(rc, "mplb_set_step_many_graphs")


def mplb_copy_probe(src, dst, nbytes, kind=0, stream=None):
    """Device copy with 16-byte accesses (bandwidth reference); src, dst are torch tensors.
    kind 0: one element per thread and round; 1: the same with non-temporal stores; 2: four
    elements per thread and round, non-temporal loads and stores; 3: each block streams its own
    contiguous 256 KB chunk."""
    import torch
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = lib().mplb_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), C.c_size_t(nbytes),
                               C.c_int(int(kind)), C.c_void_p(int(s)))
    if rc:
        raise MplbError(rc, "mplb_copy_probe")


def from_workload(w, precision="f64", arena=None):
    """A lattice set up and initialised from a workloads.Workload."""
    mode = (MPLB_COUPLED_Q19 if getattr(w, "nse_q", 15) == 19 else MPLB_COUPLED) if w.coupled else MPLB_CHE_ONLY
    lt = Lattice(w.shape, w.bc, precision, mode, w.params, arena=arena)
    if not w.coupled:
        v = w.velocity or {"kind": "zero"}
        lt.set_velocity(v["kind"], v.get("field"), v.get("U", 0.0), v.get("T", 1.0))
    lt.init(w.phi0, w.u0 if w.coupled else None)
    return lt
