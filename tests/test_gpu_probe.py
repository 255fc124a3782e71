"""The bandwidth reference copy (mplb_copy_probe) copies exactly, for every
kind, on a size with whole rounds and a tail and on one below a round."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("elems", [37, (1 << 24) + 37])
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
