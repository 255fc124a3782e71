"""The C-ABI library loads and exports every entry point its header declares
(CPU only: no call here touches a GPU)."""
import ctypes as C
import os
import subprocess

import pytest

from paper_1507_07294_amd import mplb


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mplb.LIB_PATH):
        from paper_1507_07294_amd import build
        build.build()
    return mplb.lib()


def test_exports_every_declared_symbol(lib):
    declared = mplb.declared_symbols()
    assert len(declared) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", mplb.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {line.split()[-1] for line in out.stdout.splitlines() if " T " in line}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(lib, s)


def test_host_only_calls(lib):
    assert lib.mplb_strerror(mplb.MPLB_E_NONFINITE).decode() == "non-finite population"
    n = C.c_size_t(0)
    assert lib.mplb_required_bytes(32, 32, 32, mplb.MPLB_F64, mplb.MPLB_COUPLED, C.byref(n)) == 0
    # two time levels of 22 FP64 populations plus history, phi, mu, read-out
    assert n.value >= 32 ** 3 * 8 * (2 * 22 + 3 + 2 + 1)
    m = C.c_size_t(0)
    assert lib.mplb_required_bytes(32, 32, 32, mplb.MPLB_F32_F16, mplb.MPLB_COUPLED, C.byref(m)) == 0
    assert m.value < n.value / 2
    assert lib.mplb_required_bytes(0, 32, 32, mplb.MPLB_F64, mplb.MPLB_COUPLED, C.byref(n)) == mplb.MPLB_E_INVAL
    assert lib.mplb_required_bytes(32, 32, 32, 7, mplb.MPLB_COUPLED, C.byref(n)) == mplb.MPLB_E_INVAL
    assert lib.mplb_required_bytes(1 << 11, 1 << 11, 1 << 11, 0, 0, C.byref(n)) == mplb.MPLB_E_INVAL
    # D3Q19: four more population arrays per level than D3Q15, in every
    # storage precision (16 bit: four more 2-byte arrays)
    q, r = C.c_size_t(0), C.c_size_t(0)
    assert lib.mplb_required_bytes(32, 32, 32, mplb.MPLB_F64, mplb.MPLB_COUPLED, C.byref(r)) == 0
    assert lib.mplb_required_bytes(32, 32, 32, mplb.MPLB_F64, mplb.MPLB_COUPLED_Q19, C.byref(q)) == 0
    assert q.value >= r.value + 2 * 4 * 32 ** 3 * 8
    assert lib.mplb_required_bytes(32, 32, 32, mplb.MPLB_F32, mplb.MPLB_COUPLED, C.byref(r)) == 0
    assert lib.mplb_required_bytes(32, 32, 32, mplb.MPLB_F32, mplb.MPLB_COUPLED_Q19, C.byref(q)) == 0
    extra32 = q.value - r.value
    for prec in (mplb.MPLB_F32_F16, mplb.MPLB_F32_BF16):
        assert lib.mplb_required_bytes(32, 32, 32, prec, mplb.MPLB_COUPLED, C.byref(r)) == 0
        assert lib.mplb_required_bytes(32, 32, 32, prec, mplb.MPLB_COUPLED_Q19, C.byref(q)) == 0
        assert abs((q.value - r.value) - extra32 / 2) <= 2 * 256  # the same four arrays at 2 bytes


def test_read_diagonal_rejects_bad_arguments_before_any_device_call(lib):
    out = (C.c_double * 4)()
    assert lib.mplb_read_diagonal(None, mplb.MPLB_PHI, out) == mplb.MPLB_E_INVAL
    h = C.c_void_p(1)  # never dereferenced: the field check comes first
    assert lib.mplb_read_diagonal(h, 99, out) == mplb.MPLB_E_INVAL
    assert lib.mplb_read_diagonal(h, mplb.MPLB_PHI, None) == mplb.MPLB_E_INVAL


def test_size_limit_boundary(lib):
    """The kernels index a lattice with 32-bit node offsets: just under 2^31
    nodes is accepted (here in 16-bit storage, which fits one GPU's HBM),
    exactly 2^31 is refused, as is a plane of 2^29 nodes (in-plane byte
    offsets of up to 8-byte elements must fit 32 bits)."""
    n = C.c_size_t(0)
    assert lib.mplb_required_bytes(2048, 1024, 1023, mplb.MPLB_F32_F16, mplb.MPLB_COUPLED, C.byref(n)) == 0
    assert 2048 * 1024 * 1023 * 100 < n.value < 300 * 2 ** 30
    assert lib.mplb_required_bytes(2048, 1024, 1024, mplb.MPLB_F32_F16, mplb.MPLB_COUPLED,
                                   C.byref(n)) == mplb.MPLB_E_INVAL
    assert lib.mplb_required_bytes(1 << 15, 1 << 14, 1, mplb.MPLB_F32, mplb.MPLB_COUPLED,
                                   C.byref(n)) == mplb.MPLB_E_INVAL


def test_size_limit_follows_the_padded_pitch(lib):
    """The limit is derived from the padded pitch between population arrays,
    which must fit a 32-bit int.  268434688 x 1 x 8 (N = 2^31 - 6144, about
    137 GB with 16-bit CHE-only storage) passes a bare node-count limit but
    its padded pitch exceeds INT_MAX: refused.  1000 x 1000 x 2147 (about
    258 GB with 16-bit storage) has a pitch that fits and is accepted; its
    totals pass strides over nodes in 64 bits, since the last node plus one
    stride of the totals grid passes INT_MAX."""
    n = C.c_size_t(0)
    assert lib.mplb_required_bytes(268434688, 1, 8, mplb.MPLB_F32_F16, mplb.MPLB_CHE_ONLY,
                                   C.byref(n)) == mplb.MPLB_E_INVAL
    assert lib.mplb_required_bytes(268434688, 1, 7, mplb.MPLB_F32_F16, mplb.MPLB_CHE_ONLY, C.byref(n)) == 0
    assert lib.mplb_required_bytes(1000, 1000, 2147, mplb.MPLB_F32_F16, mplb.MPLB_COUPLED, C.byref(n)) == 0
    assert n.value > 1000 * 1000 * 2147 * 100
    # the largest accepted node count: align_up(N, 256) + 27 * 256 <= 2^31 - 1
    pad = 27 * 256
    nmax = (2 ** 31 - 1 - pad) // 256 * 256
    assert lib.mplb_required_bytes(256, 1, nmax // 256, mplb.MPLB_F32_F16, mplb.MPLB_CHE_ONLY, C.byref(n)) == 0
    assert lib.mplb_required_bytes(256, 1, nmax // 256 + 1, mplb.MPLB_F32_F16, mplb.MPLB_CHE_ONLY,
                                   C.byref(n)) == mplb.MPLB_E_INVAL
    h = C.c_void_p(1)
    bc = (C.c_int * 3)(0, 0, 0)
    assert lib.mplb_create(268434688, 1, 8, bc, mplb.MPLB_F32_F16, mplb.MPLB_CHE_ONLY, None, 0,
                           C.byref(h)) == mplb.MPLB_E_INVAL
    assert h.value is None


def test_step_many_and_hooks_reject_bad_arguments_before_any_device_call(lib):
    assert lib.mplb_step_many(None, 1, 1) == mplb.MPLB_E_INVAL
    assert lib.mplb_step_many_noalloc(None, 1, 1) == mplb.MPLB_E_INVAL
    arr = (C.c_void_p * 1)(None)
    assert lib.mplb_step_many(arr, 1, 1) == mplb.MPLB_E_INVAL
    assert lib.mplb_step_many_noalloc(arr, 1, 1) == mplb.MPLB_E_INVAL
    assert lib.mplb_step_many(arr, 0, 5) == 0 and lib.mplb_step_many_noalloc(arr, 0, 5) == 0
    assert lib.mplb_check_finite(None) == mplb.MPLB_E_INVAL
    assert lib.mplb_force_tile_rows(None, 8) == mplb.MPLB_E_INVAL


def test_invalid_create_is_rejected_before_any_device_call(lib):
    h = C.c_void_p(1)
    bc = (C.c_int * 3)(0, 0, 5)
    assert lib.mplb_create(4, 4, 4, bc, 0, 0, None, 0, C.byref(h)) == mplb.MPLB_E_INVAL
    assert h.value is None
    bc = (C.c_int * 3)(0, 0, 1)
    assert lib.mplb_create(4, -1, 4, bc, 0, 0, None, 0, C.byref(h)) == mplb.MPLB_E_INVAL
    assert lib.mplb_create(4, 4, 4, bc, 0, 9, None, 0, C.byref(h)) == mplb.MPLB_E_INVAL


def test_product_path_has_no_cpu_fallback():
    """The binding never imports the oracle and refuses to run without a GPU."""
    src = open(mplb.__file__).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError):
            mplb.Lattice((4, 4, 4))


def test_binding_uses_a_single_hip_runtime():
    """torch's bundled HIP runtime and the system one share a soname; the
    binding loads torch first so that libmplb binds to torch's copy and only
    one runtime is mapped (a second one would not see torch's device state).
    Checked in a fresh process where nothing has loaded torch yet."""
    import sys
    REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1507_07294_amd import mplb\n"
            "mplb.mplb_required_bytes(8, 8, 8, mplb.MPLB_F32, mplb.MPLB_COUPLED)\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "print(len({l.split()[-1] for l in maps if 'amdhip64' in l}))\n") % REPO
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_copy_probe_rejects_bad_arguments_before_any_device_call(lib):
    fake = C.c_void_p(4096)
    assert lib.mplb_copy_probe(fake, fake, C.c_size_t(64), 4, None) == mplb.MPLB_E_INVAL
    assert lib.mplb_copy_probe(fake, fake, C.c_size_t(64), -1, None) == mplb.MPLB_E_INVAL
    assert lib.mplb_copy_probe(fake, fake, C.c_size_t(60), 0, None) == mplb.MPLB_E_INVAL
    assert lib.mplb_copy_probe(None, fake, C.c_size_t(64), 0, None) == mplb.MPLB_E_INVAL
