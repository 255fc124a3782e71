"""The bandwidth reference copy (mplb_copy_probe) copies exactly, for every
kind, on a size with whole rounds and a tail and on one below a round."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("elems", [37, (1 << 24) + 37, 3 * 16384])
def test_copy_probe_is_exact(kind, elems):
    import torch
    from paper_1507_07294_amd import mplb
    print(f"\n[case] copy probe kind={kind} elems={elems}", flush=True)
    n = elems * 4  # 16-byte elements as int32 quads
    a = torch.arange(n, dtype=torch.int32, device="cuda")
    b = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    mplb.mplb_copy_probe(a, b, n * 4, kind)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_time_stages_advances_like_step():
    """mplb_time_stages advances the state bit for bit as mplb_step does and
    reports the step kernels' time (no separate phi or mu passes)."""
    import numpy as np
    from paper_1507_07294_amd import mplb, workloads as wl
    print("\n[case] time_stages 20x18x16 f32", flush=True)
    w = wl.perturbed_case((20, 18, 16), (0, 0, 1), 91, coupled=True)
    a, b = mplb.from_workload(w, "f32"), mplb.from_workload(w, "f32")
    ms = a.time_stages(5)
    b.step(5)
    assert a.step_count == b.step_count == 5
    for k in ("phi", "ux", "p"):
        assert np.array_equal(a.read(k), b.read(k)), k
    assert ms[0] == 0.0 and ms[1] == 0.0 and ms[2] > 0.0 and ms[3] == ms[2]
    a.destroy()
    b.destroy()
