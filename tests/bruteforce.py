"""Brute-force NumPy step of the model in velocity space, written
independently of the C oracle to pin it (test helper, not a test module).

It reads the velocity tables and M from the golden fixtures, builds Gamma
from d'Humieres' polynomial basis evaluated on the Eq. 23 velocities, and
applies the collision as dense velocity-space operators:
    f* = f - (M^-1 S^f M)(f - f^eq) + M^-1 (I - S^f/2) M R         (Eqs. 4, 11)
    g* = g - (Gamma^-1 S^g Gamma)(g - g^eq) + Gamma^-1 (I - S^g/2) mT  (Eqs. 20, 27, 32)
with f^eq (Eq. 5), R (Eq. 12) and g^eq (Eqs. 21-22) in velocity space, the
stencils of Eqs. 35-36 by array shifts, and streaming by np.roll with
half-way bounce-back on wall axes.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def velocities7():
    return load_matrix("eq06_velocities_d3q7.txt").T.astype(int)  # (7, 3)


def velocities15():
    return load_matrix("eq23_velocities_d3q15.txt").T.astype(int)  # (15, 3)


def weights7(A):
    return np.array([1 - 3 * A] + [A / 2] * 6)


def weights15():
    return np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)


def velocities19():
    return load_matrix("d3q19_velocities.txt").T.astype(int)  # (19, 3)


def weights19():
    return np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def gamma19_polynomial(c):
    """d'Humieres et al. (2002) D3Q19 basis on velocities c."""
    cx, cy, cz = c[:, 0].astype(float), c[:, 1].astype(float), c[:, 2].astype(float)
    c2 = cx * cx + cy * cy + cz * cz
    rows = [np.ones_like(cx), 19 * c2 - 30, (21 * c2 * c2 - 53 * c2 + 24) / 2,
            cx, (5 * c2 - 9) * cx, cy, (5 * c2 - 9) * cy, cz, (5 * c2 - 9) * cz,
            3 * cx * cx - c2, (3 * c2 - 5) * (3 * cx * cx - c2), cy * cy - cz * cz,
            (3 * c2 - 5) * (cy * cy - cz * cz), cx * cy, cy * cz, cx * cz,
            (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz]
    return np.array(rows)


def matrix_M():
    return load_matrix("eq09_M_d3q7.txt")


def gamma_polynomial(c):
    """d'Humieres' D3Q15 basis (the polynomials behind Eq. 25) on velocities c."""
    cx, cy, cz = c[:, 0].astype(float), c[:, 1].astype(float), c[:, 2].astype(float)
    c2 = cx * cx + cy * cy + cz * cz
    rows = [np.ones_like(cx), c2 - 2, (15 * c2 * c2 - 55 * c2 + 32) / 2, cx, (5 * c2 - 13) * cx / 2,
            cy, (5 * c2 - 13) * cy / 2, cz, (5 * c2 - 13) * cz / 2, 3 * cx * cx - c2, cy * cy - cz * cz,
            cx * cy, cy * cz, cx * cz, cx * cy * cz]
    return np.array(rows)


def opposite(c):
    return np.array([int(np.where((c == -c[i]).all(axis=1))[0][0]) for i in range(len(c))])


class Brute:
    def __init__(self, shape, bc, params, coupled=True, u_field=None, q=15):
        self.nx, self.ny, self.nz = shape
        self.bc = bc
        self.p = params
        self.coupled = coupled
        self.u_field = u_field  # (3, nz, ny, nx) prescribed velocity for CHE-only
        A = params.A
        self.c7, self.w7, self.cs2f = velocities7(), weights7(A), A
        self.c15, self.w15, self.cs2 = velocities15(), weights15(), 1.0 / 3.0
        self.q = q
        # lattice of the g populations (the stencils keep the D3Q15 weights)
        self.cg, self.wg = (velocities19(), weights19()) if q == 19 else (self.c15, self.w15)
        self.M = matrix_M()
        self.Gm = gamma19_polynomial(self.cg) if q == 19 else gamma_polynomial(self.c15)
        self.Minv = np.linalg.inv(self.M)
        self.Ginv = np.linalg.inv(self.Gm)
        self.opp7, self.opp15 = opposite(self.c7), opposite(self.cg)
        self.beta = 3 * params.sigma / (4 * params.width)
        self.kappa = 3 * params.width * params.sigma / 8
        tau_f = 1 / params.s_f[1]
        self.eta = params.mobility / (A * (tau_f - 0.5))
        tau_g = 3 * params.nu + 0.5
        self.stencil7 = getattr(params, "stencil", 0) == 1
        self.forcing28 = getattr(params, "forcing", 0) == 1
        if getattr(params, "lambda_override", 0):
            tau_g = 1 / params.lambda_g[9]
        if q == 19:  # stress moments at 1/tau_g, the rest at 1
            lam = np.ones(19)
            lam[[9, 11, 13, 14, 15]] = 1 / tau_g
        else:
            lam = np.array(params.lambda_g, dtype=float)
            lam[9:14] = 1 / tau_g
        self.Sf = np.diag(params.s_f)
        self.Sg = np.diag(lam)
        I7, I15 = np.eye(7), np.eye(q)
        self.Kf = self.Minv @ self.Sf @ self.M
        self.Rf = self.Minv @ (I7 - self.Sf / 2) @ self.M
        self.Kg = self.Ginv @ self.Sg @ self.Gm
        self.Hg = self.Ginv @ (I15 - self.Sg / 2)

    # ---- Eqs. 35-36 by shifts of a ghost-padded array ----
    def _pad(self, chi):
        out = chi
        for ax, a in ((2, 0), (1, 1), (0, 2)):
            mode = "edge" if self.bc[a] == 1 else "wrap"
            pw = [(0, 0)] * 3
            pw[ax] = (1, 1)
            out = np.pad(out, pw, mode=mode)
        return out

    def _nb(self, padded, c):
        nz, ny, nx = self.nz, self.ny, self.nx
        return padded[1 + c[2]:1 + c[2] + nz, 1 + c[1]:1 + c[1] + ny, 1 + c[0]:1 + c[0] + nx]

    def _stencil(self):
        """velocities, weights, c_s^2 of the finite differences (Eqs. 35-36)"""
        if self.stencil7:
            return self.c7, self.w7, self.cs2f
        return self.c15, self.w15, self.cs2

    def grad(self, chi):
        c, w, cs2 = self._stencil()
        P = self._pad(chi)
        out = np.zeros((3,) + chi.shape)
        for i in range(1, len(c)):
            v = self._nb(P, c[i])
            for a in range(3):
                out[a] += w[i] * c[i][a] * v / cs2
        return out

    def lap(self, chi):
        c, w, cs2 = self._stencil()
        P = self._pad(chi)
        out = np.zeros(chi.shape)
        for i in range(1, len(c)):
            out += 2 * w[i] * (self._nb(P, c[i]) - chi) / cs2
        return out

    # ---- one step ----
    def macro(self, f, g, n):
        p = self.p
        phi = f.sum(axis=0)
        rho = (1 + phi) / 2 * p.rho_l + (1 - phi) / 2 * p.rho_g
        mu = 4 * self.beta * phi * (phi ** 2 - 1) - self.kappa * self.lap(phi)
        if not self.coupled:
            u = np.zeros((3,) + phi.shape) if self.u_field is None else self.u_field.copy()
            return dict(phi=phi, rho=rho, mu=mu, u=u, p=np.zeros_like(phi), F=np.zeros_like(u),
                        grho=np.zeros_like(u))
        gphi = self.grad(phi)
        grho = self.grad(rho)
        lmu = self.lap(mu)
        Fs = mu * gphi
        G = np.stack([(rho - p.rho_ref) * p.gravity[a] for a in range(3)])
        j = np.einsum("ia,i...->a...", self.cg.astype(float), g)
        dr = p.rho_l - p.rho_g
        u = (j + 0.5 * (Fs + G)) / (rho - 0.25 * dr * p.mobility * lmu)
        F = Fs + 0.5 * dr * p.mobility * lmu * u + G
        uu = (u ** 2).sum(axis=0)
        s0 = self.wg[0] * (-uu / (2 * self.cs2))
        pr = self.cs2 / (1 - self.wg[0]) * (g[1:].sum(axis=0) + 0.5 * (u * grho).sum(axis=0) + rho * s0)
        return dict(phi=phi, rho=rho, mu=mu, u=u, p=pr, F=F, grho=grho)

    def feq(self, phi, mu, u):
        out = np.empty((7,) + phi.shape)
        out[0] = phi + (self.w7[0] - 1) * self.eta * mu
        for i in range(1, 7):
            cu = sum(self.c7[i][a] * phi * u[a] for a in range(3))
            out[i] = self.w7[i] * self.eta * mu + self.w7[i] * cu / self.cs2f
        return out

    def R(self, dphiu):
        out = np.empty((7,) + dphiu.shape[1:])
        for i in range(7):
            out[i] = self.w7[i] * sum(self.c7[i][a] * dphiu[a] for a in range(3)) / self.cs2f
        return out

    def s_i(self, u):
        """s_i(u) of Eq. 22 for every velocity of the g lattice."""
        uu = (u ** 2).sum(axis=0)
        out = np.empty((self.q,) + uu.shape)
        for i in range(self.q):
            cu = sum(self.cg[i][a] * u[a] for a in range(3))
            out[i] = self.wg[i] * (cu / self.cs2 + cu ** 2 / (2 * self.cs2 ** 2) - uu / (2 * self.cs2))
        return out

    def geq(self, pr, rho, u):
        s = self.s_i(u)
        out = np.empty((self.q,) + pr.shape)
        for i in range(self.q):
            out[i] = pr / self.cs2 * (self.wg[i] - (1.0 if i == 0 else 0.0)) + rho * s[i]
        return out

    def T(self, u, grho, F):
        """Eq. 28 in velocity space."""
        s = self.s_i(u)
        out = np.zeros((self.q,) + u.shape[1:])
        for i in range(self.q):
            for a in range(3):
                out[i] += (self.cg[i][a] - u[a]) * (s[i] * grho[a] * self.cs2 + F[a] * (s[i] + self.wg[i]))
        return out / self.cs2

    def mT(self, u, grho, F):
        """Eq. 32 (c = 1)."""
        cs2 = self.cs2
        a = grho * cs2 + F
        ugr = (u * grho).sum(axis=0)
        uF = (u * F).sum(axis=0)
        z = np.zeros_like(ugr)
        return np.stack([ugr, -ugr * cs2 + 2 * uF, -(7 * ugr * cs2 + 10 * uF), F[0], -7 * F[0] / 3,
                         F[1], -7 * F[1] / 3, F[2], -7 * F[2] / 3,
                         4 * u[0] * a[0] - 2 * u[1] * a[1] - 2 * u[2] * a[2],
                         2 * u[1] * a[1] - 2 * u[2] * a[2], u[0] * a[1] + u[1] * a[0],
                         u[1] * a[2] + u[2] * a[1], u[0] * a[2] + u[2] * a[0], z])

    def _stream(self, post, c, opp):
        new = np.zeros_like(post)
        coords = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        n_ax = (self.nx, self.ny, self.nz)
        for i in range(len(c)):
            leave = np.zeros(post.shape[1:], dtype=bool)
            for a in range(3):
                if self.bc[a] == 1 and c[i][a] != 0:
                    q = coords[2 - a] + c[i][a]
                    leave |= (q < 0) | (q >= n_ax[a])
            new[opp[i]] += np.where(leave, post[i], 0.0)
            stay = np.where(leave, 0.0, post[i])
            new[i] += np.roll(stay, shift=(c[i][2], c[i][1], c[i][0]), axis=(0, 1, 2))
        return new

    def step(self, f, g, phiu_prev, n=0):
        m = self.macro(f, g, n)
        phiu = m["phi"] * m["u"]
        dphiu = phiu - phiu_prev
        fe = self.feq(m["phi"], m["mu"], m["u"])
        Rv = self.R(dphiu)
        fpost = f - np.einsum("ij,j...->i...", self.Kf, f - fe) + np.einsum("ij,j...->i...", self.Rf, Rv)
        f_new = self._stream(fpost, self.c7, self.opp7)
        if not self.coupled:
            return f_new, g, phiu
        ge = self.geq(m["p"], m["rho"], m["u"])
        if self.q == 19 or self.forcing28:  # Gamma T of Eq. 28, untruncated
            mt = np.einsum("ij,j...->i...", self.Gm, self.T(m["u"], m["grho"], m["F"]))
        else:
            mt = self.mT(m["u"], m["grho"], m["F"])
        gpost = g - np.einsum("ij,j...->i...", self.Kg, g - ge) + np.einsum("ij,j...->i...", self.Hg, mt)
        g_new = self._stream(gpost, self.cg, self.opp15)
        return f_new, g_new, phiu

    def init(self, phi0, u0=None):
        """Equilibrium start: f = f^eq(phi0, mu0, u0), g = g^eq(p = 0), (phi u)_prev = phi0 u0."""
        u = np.zeros((3,) + phi0.shape) if u0 is None else u0
        if not self.coupled:
            u = np.zeros((3,) + phi0.shape) if self.u_field is None else self.u_field
        mu = 4 * self.beta * phi0 * (phi0 ** 2 - 1) - self.kappa * self.lap(phi0)
        rho = (1 + phi0) / 2 * self.p.rho_l + (1 - phi0) / 2 * self.p.rho_g
        f = self.feq(phi0, mu, u)
        g = self.geq(np.zeros_like(phi0), rho, u) if self.coupled else np.zeros((self.q,) + phi0.shape)
        return f, g, phi0 * u
