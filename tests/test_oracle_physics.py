"""Physics pins of the oracle (CPU only): the oracle must reproduce what the
Chapman-Enskog relations of the paper and textbook interface physics fix."""
import numpy as np
import pytest

import oracle.orc as orc
from paper_1507_07294_amd import workloads as wl


@pytest.mark.parametrize("tau_g", [0.6, 0.8, 1.0])
def test_shear_wave_viscosity(tau_g):
    """nu = c_s^2 (tau_g - 1/2) (Eq. 33): a shear wave u_x = U sin(qz) in one
    phase decays as exp(-nu q^2 t)."""
    nu, L = (tau_g - 0.5) / 3, 64
    p = wl.ModelParams(sigma=0.01, width=4.0, mobility=0.1, nu=nu)
    z = np.arange(L)[:, None, None] * np.ones((L, 2, 2))
    u0 = np.zeros((3, L, 2, 2))
    u0[0] = 1e-3 * np.sin(2 * np.pi * z / L)
    o = orc.Oracle((2, 2, L), (0, 0, 0), orc.COUPLED, p)
    o.init(np.ones((L, 2, 2)), u0)
    basis = np.sin(2 * np.pi * z / L)

    def amp():
        return (o.read("ux") * basis).sum() / (basis * basis).sum()

    o.step(100)
    a1 = amp()
    o.step(500)
    a2 = amp()
    q = 2 * np.pi / L
    assert abs(np.log(a1 / a2) / (q * q * 500) / nu - 1) < 5e-3


@pytest.mark.parametrize("L", [32, 64])
def test_mobility_decay(L):
    """M = eta c_s^2 (tau_f - 1/2) (Eq. 19): with u = 0 a small mode
    phi = 1 + e cos(qx) decays at M s (8 beta + k s), s = 2(1 - cos q) the
    symbol of the Laplacian (linearised Eqs. 1-2)."""
    sigma, D, M = 0.04, 2.0, 0.1
    p = wl.ModelParams(sigma=sigma, width=D, mobility=M, s_f=wl.SF_ZALESAK, nu=0.1)
    x = np.arange(L)[None, None, :] * 1.0
    o = orc.Oracle((L, 1, 1), (0, 0, 0), orc.CHE_ONLY, p)
    o.set_velocity(orc.VEL_ZERO)
    o.init(1 + 1e-3 * np.cos(2 * np.pi * x / L))
    basis = np.cos(2 * np.pi * x / L)

    def amp():
        return ((o.read("phi") - 1) * basis).sum() / (basis * basis).sum()

    o.step(200)
    a1 = amp()
    o.step(2000)
    a2 = amp()
    beta, k = 3 * sigma / (4 * D), 3 * D * sigma / 8
    s = 2 * (1 - np.cos(2 * np.pi / L))
    assert abs(np.log(a1 / a2) / 2000 / (M * s * (8 * beta + k * s)) - 1) < 0.02


def test_flat_interface_is_stationary():
    """phi = tanh(2 z / D) is the equilibrium profile of Eq. 2 with
    k/beta = D^2/2; between no-slip walls a flat interface stays put, with no
    flow, and keeps its profile (Eqs. 42-43 with h = 0 and no gravity)."""
    nz, D = 64, 4.0
    p = wl.ModelParams(sigma=0.01, width=D, rho_l=3.0, rho_g=1.0, mobility=0.1, nu=0.1)
    zc = np.arange(nz) + 0.5
    prof = np.tanh(2 * (zc - nz / 2) / D)
    o = orc.Oracle((4, 4, nz), (0, 0, 1), orc.COUPLED, p)
    o.init(np.broadcast_to(prof[:, None, None], (nz, 4, 4)).copy())
    o.step(2000)
    phi = o.read("phi")[:, 0, 0]
    i = int(np.where(np.diff(np.sign(phi)))[0][0])
    zcross = zc[i] - phi[i] / (phi[i + 1] - phi[i])
    assert abs(zcross - nz / 2) < 1e-3
    assert max(np.abs(o.read(k)).max() for k in ("ux", "uy", "uz")) < 1e-5
    assert np.abs(phi - prof).max() < 0.02


def test_laplace_law_static_droplet():
    """Static droplet, 32^3, R = 8, D = 4, sigma = 0.01, density ratio 3, 500
    steps: the pressure jump matches 2 sigma / R_eff within 5 %."""
    w = wl.static_droplet()
    o = orc.Oracle(w.shape, w.bc, orc.COUPLED, w.params)
    o.init(w.phi0)
    t0 = o.totals()[0]
    o.step(w.steps)
    assert abs(o.totals()[0] - t0) < 1e-12 * np.abs(w.phi0).sum()
    pr, phi = o.read("p"), o.read("phi")
    n = 32
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((xx - 16.0) ** 2 + (yy - 16.0) ** 2 + (zz - 16.0) ** 2)
    R_eff = (3 * ((1 + phi) / 2).sum() / (4 * np.pi)) ** (1 / 3)
    dp = pr[r < 8 - 4].mean() - pr[r > 8 + 4].mean()
    assert abs(dp / (2 * w.params.sigma / R_eff) - 1) < 0.05
