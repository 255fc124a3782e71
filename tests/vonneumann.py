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

The second part linearises the whole coupled step (both lattices) about a
uniform bulk state by impulse responses of the NumPy step of bruteforce.py.
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


# ---------------------------------------------------------------------------
# The coupled step (Eqs. 4 and 20 with Eqs. 28-36) linearised about a uniform
# bulk state, from the independent NumPy step of bruteforce.py.  On a
# periodic box a uniform state (phi_b, u, p = 0, G = 0 with rho_ref the bulk
# density) is a fixed point and the step is the same at every node, so its
# linearisation is diagonal in Fourier space: the response to a unit impulse
# in state component j at node 0 is, after an FFT over the box, column j of
# G(k) for every wave vector k at once.  The state of a node is the 7 f, the
# 15 g and the 3 words of (phi u) of the previous level.
# ---------------------------------------------------------------------------

def coupled_base(params, shape, phi_b, u):
    """The uniform state (f, g, (phi u)_prev) of the NumPy step."""
    nx, ny, nz = shape
    B = bf.Brute(shape, (0, 0, 0), params, coupled=True)
    uf = np.stack([np.full((nz, ny, nx), float(v)) for v in u])
    f, g, pu = B.init(np.full((nz, ny, nx), float(phi_b)), uf)
    return B, np.concatenate([f, g, pu])


def coupled_step_matrices(params, shape, phi_b, u, eps=1e-7):
    """G(k) of the coupled step on a periodic box, shape (nz, ny, nx, 25, 25),
    by central differences of impulse responses, and the base state."""
    nx, ny, nz = shape
    B, base = coupled_base(params, shape, phi_b, u)
    D = base.shape[0]
    G = np.zeros((D, D, nz, ny, nx), dtype=complex)
    for j in range(D):
        r = []
        for s in (1.0, -1.0):
            st = base.copy()
            st[j, 0, 0, 0] += s * eps
            fa, ga, pa = B.step(st[:7], st[7:22], st[22:])
            r.append(np.concatenate([fa, ga, pa]))
        G[:, j] = np.fft.fftn((r[0] - r[1]) / (2 * eps), axes=(1, 2, 3))
    return np.moveaxis(G, (0, 1), (-2, -1)), base


def coupled_largest_growth(params, shape, phi_b, u):
    """(max |lambda| over the box's wave vectors, its (kz, ky, kx) index, G)."""
    G, _ = coupled_step_matrices(params, shape, phi_b, u)
    lam = np.abs(np.linalg.eigvals(G.reshape(-1, G.shape[-1], G.shape[-1]))).max(axis=1)
    idx = np.unravel_index(int(lam.argmax()), G.shape[:3])
    return float(lam.max()), idx, G
