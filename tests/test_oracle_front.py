"""Pins of the oracle's interface-extreme diagnostic (spike tip and bubble
front of a layered run, Sec. III C): profiles whose zero crossings are known
in closed form.  At step 0, phi = sum_i f_i^eq = phi_0 (Eq. 5 sums to phi),
so the crossings are those of the initial field."""
import numpy as np

import oracle.orc as orc
from paper_1507_07294_amd import workloads as wl


def _oracle(phi0, bc=(0, 0, 1)):
    nz, ny, nx = phi0.shape
    p = wl.ModelParams(sigma=0.0, width=4.0, mobility=0.05, s_f=wl.SF_RT, nu=0.1)
    o = orc.Oracle((nx, ny, nz), bc, orc.COUPLED, p)
    o.init(phi0)
    return o


def test_linear_columns_cross_at_their_centres():
    """phi linear in z with a column-dependent zero: linear interpolation is
    exact, so the extremes are the extreme column zeros."""
    nx, ny, nz = 12, 10, 24
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None] + 0.5  # layer k at k + 1/2
    zc = 11.3 + 2.1 * np.cos(2 * np.pi * x / nx) + 1.4 * np.sin(2 * np.pi * y / ny)
    phi0 = np.broadcast_to((z - zc) / 7.0, (nz, ny, nx)).copy()
    lo, hi = _oracle(phi0).front()
    assert abs(lo - zc.min()) < 1e-12 and abs(hi - zc.max()) < 1e-12


def test_slab_between_two_interfaces():
    """A heavy slab on layers 5..9: sign changes midway between layers 4, 5
    and 9, 10, i.e. at z = 5 and z = 10 (layer k at k + 1/2)."""
    nx, ny, nz = 4, 3, 16
    phi0 = -np.ones((nz, ny, nx))
    phi0[5:10] = 1.0
    lo, hi = _oracle(phi0).front()
    assert lo == 5.0 and hi == 10.0


def test_no_interface():
    lo, hi = _oracle(np.full((8, 4, 4), 0.5)).front()
    assert lo == -1.0 and hi == -1.0


def test_rayleigh_taylor_initial_front():
    """The Rayleigh-Taylor layer of Eq. 43 starts with its interface at
    2W + h, h between -0.1 W (spike, x = y = W/2) and +0.1 W (bubble,
    x = y = 0); tanh is odd about its zero, so interpolation is close."""
    W = 16
    w = wl.rayleigh_taylor(W=W, Re=256.0)
    o = orc.Oracle(w.shape, w.bc, orc.COUPLED, w.params)
    o.init(w.phi0)
    lo, hi = o.front()
    assert abs(lo - (2 * W - 0.1 * W)) < 0.02 and abs(hi - (2 * W + 0.1 * W)) < 0.02
