"""Linear (von Neumann) analysis of the D3Q7 MRT step for the
Cahn-Hilliard equation about a uniform bulk phase under a uniform flow (test
helper, not a test module; independent of the C oracle).

About phi = phi_b (|phi_b| = 1, so mu = 0, Eq. 2) and a constant prescribed u,
a perturbation proportional to exp(i q.x) evolves linearly.  Its state is the
seven f_i and phi of the previous level, which enters the time derivative of
phi u by the backward difference of Eq. 34.  One step, for one wave vector q:

    phi'   = sum_i f'_i                                          (Eq. 13)
    mu'    = 4 beta (3 phi_b^2 - 1) phi' - kappa L(q) phi'       (Eq. 2; L the
             symbol of the isotropic Laplacian of Eq. 36 on the D3Q15 weights)
    f^eq'  = Eq. 5 linearised: rest phi' + (w_0 - 1) eta mu',
             moving w_i eta mu' + w_i c_i.u phi' / c_s^2
    R'     = w_i c_i.u (phi' - phi'_prev) / c_s^2                (Eqs. 12, 34)
    f*     = f' - (M^-1 S M)(f' - f^eq') + M^-1 (I - S/2) M R'    (Eqs. 4, 11)
    f'(n+1)_i = f*_i exp(-i q.c_i)                                (Eq. 16, pull)
    phi'_prev(n+1) = phi'(n)

so the step is an 8 x 8 complex matrix G(q).  The velocity tables, M and the
weights come from the golden fixtures of the printed equations.
"""
from __future__ import annotations

import numpy as np

import bruteforce as bf


def laplacian_symbol(q):
    """Eq. 36 on exp(i q.x) with the D3Q15 weights (c_s^2 = 1/3)."""
    c, w = bf.velocities15(), bf.weights15()
    return float(sum(2 * w[i] * (np.cos(q @ c[i]) - 1) * 3.0 for i in range(1, 15)))


def coefficients(sigma, D, mobility, s_f, A=0.25):
    """beta, kappa (after Eq. 2) and eta (Eq. 19 with c_s^2 = A, tau_f = 1/s_1)."""
    beta = 3 * sigma / (4 * D)
    kappa = 3 * D * sigma / 8
    eta = mobility / (A * (1 / s_f[1] - 0.5))
    return beta, kappa, eta


def step_matrix(q, u, sigma, D, mobility, s_f, phi_b=1.0, A=0.25, source=True):
    """G(q): the linearised step acting on (f'_0..f'_6, phi'_prev)."""
    q = np.asarray(q, dtype=float)
    u = np.asarray(u, dtype=float)
    c, w = bf.velocities7(), bf.weights7(A)
    M = bf.matrix_M()
    Mi = np.linalg.inv(M)
    S = np.diag(np.asarray(s_f, dtype=float))
    beta, kappa, eta = coefficients(sigma, D, mobility, s_f, A)
    dmu = 4 * beta * (3 * phi_b ** 2 - 1) - kappa * laplacian_symbol(q)  # d mu / d phi for this mode
    cu = c @ u
    coll = np.eye(7) - Mi @ S @ M
    src = Mi @ (np.eye(7) - S / 2) @ M
    shift = np.exp(-1j * (c @ q))
    G = np.zeros((8, 8), dtype=complex)
    for j in range(8):
        e = np.zeros(8)
        e[j] = 1.0
        f, phi_prev = e[:7], e[7]
        phi = f.sum()
        mu = dmu * phi
        feq = w * eta * mu + w * cu * phi / A
        feq[0] = phi + (w[0] - 1) * eta * mu
        R = w * cu * (phi - phi_prev) / A if source else np.zeros(7)
        fs = coll @ f + (Mi @ S @ M) @ feq + src @ R
        G[:7, j] = fs * shift
        G[7, j] = phi
    return G


def spectral_radius(G):
    return float(np.abs(np.linalg.eigvals(G)).max())


def grid_wavevectors(shape):
    """Every wave vector of a periodic (nx, ny, nz) box."""
    ks = [2 * np.pi * np.fft.fftfreq(n) * 1.0 for n in shape]
    return [np.array([kx, ky, kz]) for kx in ks[0] for ky in ks[1] for kz in ks[2]]


def largest_growth(shape, u, sigma, D, mobility, s_f, source=True):
    """(max |lambda|, q) over the wave vectors of a periodic box."""
    best = (0.0, None)
    for q in grid_wavevectors(shape):
        r = spectral_radius(step_matrix(q, u, sigma, D, mobility, s_f, source=source))
        if r > best[0]:
            best = (r, q)
    return best
