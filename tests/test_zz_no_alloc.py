"""mplb_step_many_noalloc, the batched step with no device or host
allocation (its batch table is a static device array), against
mplb_step_many through the C-ABI: bitwise the same fields on two calls in a
row, the second with fewer and smaller lattices, and a batch larger than the
static table is refused with a clear error."""
import numpy as np
import pytest

import helpers
from paper_1507_07294_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _unit(w):
    w.params = w.params.replace(lambda_g=(1.0,) * 15)
    return w


def _pair(ws, precision):
    return [helpers.gpu_for(w, precision) for w in ws], [helpers.gpu_for(w, precision) for w in ws]


@pytest.mark.parametrize("precision", ["f32", "f16", "f64"])
def test_noalloc_equals_step_many(precision):
    from paper_1507_07294_amd import mplb
    print(f"\n[case] step_many_noalloc vs step_many {precision}", flush=True)
    first = [_unit(wl.perturbed_case((40, 36, 30), (0, 0, 1), 201)), wl.static_droplet(n=32, R=8.0),
             wl.rayleigh_taylor(W=24, Re=256.0), _unit(wl.perturbed_case((17, 21, 15), (1, 0, 0), 202)),
             wl.static_droplet(n=48, R=12.0, ratio=5.0)]
    second = [wl.static_droplet(n=16, R=4.0, ratio=2.0), _unit(wl.perturbed_case((9, 10, 11), (1, 1, 1), 203))]
    for ws, steps in ((first, 9), (second, 6)):
        ref, got = _pair(ws, precision)
        got[0].step(1)  # different buffer parities within the batch
        ref[0].step(1)
        mplb.mplb_step_many(ref, steps)
        mplb.mplb_step_many_noalloc(got, steps)
        for w, a, b in zip(ws, ref, got):
            assert a.step_count == b.step_count
            fa, fb = helpers.fields_of(a), helpers.fields_of(b)
            for k in fa:
                assert np.array_equal(fa[k], fb[k]), (w.name, k)
        for g in ref + got:
            g.destroy()


def test_noalloc_refuses_a_batch_above_its_table():
    from paper_1507_07294_amd import mplb
    g = helpers.gpu_for(wl.static_droplet(n=8, R=2.0), "f32")
    with pytest.raises(mplb.MplbError) as ei:
        mplb.mplb_step_many_noalloc([g] * (mplb.MPLB_NOALLOC_MAX_LATTICES + 1), 1)
    assert ei.value.code == mplb.MPLB_E_INVAL
    assert "exceed" in str(ei.value) and str(mplb.MPLB_NOALLOC_MAX_LATTICES) in str(ei.value)
    assert g.step_count == 0
    g.destroy()
