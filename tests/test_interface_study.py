"""Host-side pieces of the interface-capturing studies (CPU only)."""
import numpy as np

from paper_1507_07294_amd import interface_study as ist
from paper_1507_07294_amd import workloads as wl


def test_err_eq40_closed_forms():
    """Eq. 40 is 0 for an unchanged field, 2 for a sign flip, and for a
    field shifted by a constant c on a field of constant magnitude a it is
    |c| / a."""
    rng = np.random.default_rng(3)
    phi = np.tanh(rng.normal(size=(6, 5, 4)))
    assert ist.err_eq40(phi, phi) == 0.0
    assert abs(ist.err_eq40(-phi, phi) - 2.0) < 1e-15
    a = np.full((3, 3, 3), 0.8)
    assert abs(ist.err_eq40(a + 0.1, a) - 0.125) < 1e-15


def test_srt_rates_keep_the_mobility_rate():
    """The SRT special case keeps s_1 (which sets the mobility, Eq. 19) for
    every moment."""
    assert ist.srt_rates(wl.SF_ZALESAK) == tuple([4.0 / 3.0] * 7)


def test_zalesak_revolution_length():
    """Eq. 37 rotates at U pi / n per step: one revolution is 2 n / U steps
    (10^4 at n = 100, U = 0.02, as the paper states)."""
    w = wl.zalesak(n=100)
    assert int(round(2 * 100 / w.velocity["U"])) == 10000
