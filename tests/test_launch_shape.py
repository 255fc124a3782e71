"""The launch shape of a step (mplb_launch_shape, a host computation: no GPU
needed): which kernel runs and how the lattice is split into tiles and z
segments.  The split changes only the speed of a step, never its results
(the GPU tests compare tilings bit for bit), so these tests pin the rules
themselves and the invariants every split must keep."""
import numpy as np
import pytest

from paper_1507_07294_amd import mplb

P = mplb.PRECISIONS
COUPLED, CHE, Q19 = mplb.MPLB_COUPLED, mplb.MPLB_CHE_ONLY, mplb.MPLB_COUPLED_Q19


def shape(dims, prec, mode, rows=0):
    return mplb.mplb_launch_shape(*dims, P[prec], mode, rows)


@pytest.mark.parametrize("dims,prec,mode,kind,tile,lz,blocks", [
    # the benchmark box: FP32 on 16-row tiles in two rounds of one block per
    # CU; 16-bit populations on 8-row tiles in one round of two; FP64 (one
    # block per CU) in one round of 256
    ((256, 256, 1024), "f32", COUPLED, 1, (64, 16), 128, 512),
    ((256, 256, 1024), "f16", COUPLED, 0, (64, 8), 256, 512),
    ((256, 256, 1024), "bf16", COUPLED, 0, (64, 8), 256, 512),
    ((256, 256, 1024), "f64", COUPLED, 0, (64, 8), 512, 256),
    ((256, 256, 1024), "f32", Q19, 1, (64, 16), 128, 512),
    # a lattice that cannot fill the chip: segments of 5 planes
    ((32, 32, 32), "f32", COUPLED, 0, (64, 8), 5, 28),
    ((32, 32, 32), "f64", COUPLED, 0, (64, 8), 5, 28),
    # between one and two blocks per CU: one block per CU where its march is
    # shorter (72^3: 216 blocks of 6 planes rather than 270 of 5; W = 64
    # Rayleigh-Taylor: 256 of 8 rather than 416 of 5), two where it is not
    # (96^3: 480 blocks of 5 planes)
    ((72, 72, 72), "f32", COUPLED, 0, (64, 8), 6, 216),
    ((64, 64, 256), "f32", COUPLED, 0, (64, 8), 8, 256),
    ((96, 96, 96), "f32", COUPLED, 0, (64, 8), 5, 480),
    # 16-row tiles only where they fill 512 blocks
    ((128, 128, 512), "f32", COUPLED, 1, (64, 16), 16, 512),
    ((96, 96, 384), "f32", COUPLED, 0, (64, 8), 19, 504),
    # CHE-only: two nodes per thread from 5 M nodes and 384 blocks
    ((256, 256, 256), "f32", CHE, 3, (128, 8), 32, 512),
    ((256, 256, 256), "f16", CHE, 3, (128, 8), 32, 512),
    ((176, 176, 176), "f32", CHE, 3, (128, 8), 16, 484),
    ((160, 160, 160), "f32", CHE, 2, (64, 8), 20, 480),
    ((128, 128, 128), "f32", CHE, 2, (64, 8), 8, 512),
    ((72, 72, 72), "f32", CHE, 2, (64, 8), 6, 216),
    # FP64 CHE-only: one node per thread, one round of 256 blocks
    ((256, 256, 256), "f64", CHE, 2, (64, 8), 128, 256),
    ((128, 128, 128), "f64", CHE, 2, (64, 8), 16, 256),
])
def test_rules(dims, prec, mode, kind, tile, lz, blocks):
    s = shape(dims, prec, mode)
    assert (s["kind"], s["tile"], s["lz"], s["blocks"]) == (kind, tile, lz, blocks), s


def _check_split(dims, s):
    nx, ny, nz = dims
    tw, th = s["tile"]
    tiles = -(-nx // tw) * -(-ny // th)
    assert s["blocks"] == tiles * s["segments"]
    # the segments cover the z axis exactly once: all but the last hold lz
    # planes, the last at least one
    assert s["segments"] * s["lz"] >= nz > (s["segments"] - 1) * s["lz"]
    assert 1 <= s["lz"] <= nz


def test_invariants_on_random_lattices():
    """On seeded random lattices of 1 to 3000 nodes per axis, in every
    precision and mode: the split covers the lattice exactly, the automatic
    choice never launches more than 512 blocks unless the tiles alone exceed
    that (one segment per column), FP64 never more than 256 on the same
    terms, and segments keep their minimum length (5 planes for 8-row tiles
    of a coupled lattice, 16 for 16-row tiles, 5 or 8 for the CHE-only
    kernels) unless the lattice is shorter."""
    rng = np.random.default_rng(20261206)
    checked = 0
    for _ in range(4000):
        dims = tuple(int(v) for v in np.exp(rng.uniform(0, np.log(3000), 3)).astype(int) + 1)
        if dims[0] * dims[1] * dims[2] >= 2 ** 31 - 2 ** 20:
            continue
        prec = ("f64", "f32", "f16", "bf16")[int(rng.integers(0, 4))]
        mode = (COUPLED, CHE, Q19)[int(rng.integers(0, 3))]
        s = shape(dims, prec, mode)
        _check_split(dims, s)
        tw, th = s["tile"]
        cols = -(-dims[0] // tw) * -(-dims[1] // th)
        cap = 256 if prec == "f64" else 512
        assert s["blocks"] <= max(cap, cols), (dims, prec, mode, s)
        min_lz = {0: 5, 1: 16, 2: 5, 3: 8}[s["kind"]]
        assert s["lz"] >= min(min_lz, dims[2]), (dims, prec, mode, s)
        if s["kind"] == 1:
            assert prec == "f32" and mode != CHE and s["blocks"] >= 512
        if s["kind"] == 3:
            assert prec != "f64" and mode == CHE and dims[0] * dims[1] * dims[2] >= 5_000_000
        checked += 1
    assert checked > 3000


def test_forced_rows():
    """rows = 8 or 16 selects the kernel as mplb_force_tile_rows does; 16 is
    refused where no such kernel exists."""
    assert shape((256, 256, 1024), "f32", COUPLED, rows=8)["kind"] == 0
    assert shape((64, 64, 64), "f32", COUPLED, rows=16)["kind"] == 1
    assert shape((64, 64, 64), "f16", CHE, rows=16)["kind"] == 3
    assert shape((256, 256, 256), "f32", CHE, rows=8)["kind"] == 2
    for prec, mode in (("f16", COUPLED), ("f64", COUPLED), ("f64", CHE)):
        with pytest.raises(mplb.MplbError):
            shape((64, 64, 64), prec, mode, rows=16)
    for dims, rows in (((0, 4, 4), 0), ((4, 4, 4), 12)):
        with pytest.raises(mplb.MplbError):
            shape(dims, "f32", COUPLED, rows=rows)
