"""The windowed oracle used for sampled parity at full lattice sizes equals
the oracle run on the whole lattice (CPU only)."""
import numpy as np

import helpers
from paper_1507_07294_amd import workloads as wl


def test_window_matches_full_lattice():
    shape, bc = (40, 36, 44), (0, 0, 1)
    w = wl.perturbed_case(shape, bc, 12, coupled=True)
    steps = 2
    o = helpers.oracle_for(w)
    o.step(steps)
    full = {k: o.read(k) for k in helpers.FIELDS}
    rng = np.random.default_rng(3)
    nodes = [(0, 0, 0), (39, 35, 43), (20, 18, 22), (5, 30, 1)] + \
            [tuple(int(v) for v in rng.integers(0, shape)) for _ in range(4)]
    for (x, y, z) in nodes:
        win = helpers.window_oracle_fields(w, (x, y, z), steps)
        for k in helpers.FIELDS:
            assert abs(win[k] - full[k][z, y, x]) <= 1e-15 * max(1.0, abs(full[k][z, y, x])), (k, x, y, z)
