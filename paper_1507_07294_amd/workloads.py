"""Seeded synthetic inputs shared by the GPU library's users, the tests and the
benchmark.

This module holds no arithmetic of the lattice-Boltzmann method: it builds
initial order-parameter fields, optional initial velocities and parameter
records for the workloads the paper runs (Sec. III), and the seeded serving
trace.  Arrays follow the lattice layout: a scalar field has shape
(nz, ny, nx) with x fastest; a vector field has shape (3, nz, ny, nx).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

# Relaxation sets the paper prints.
SF_ZALESAK = (1.0, 4.0 / 3.0, 4.0 / 3.0, 4.0 / 3.0, 1.2, 1.2, 1.2)  # Eq. 38 (also Sec. III B)
SF_RT = (1.0, 1.25, 1.25, 1.25, 1.2, 1.0, 1.0)  # Eq. 45


@dataclasses.dataclass
class ModelParams:
    """Physical and relaxation parameters of the model (lattice units).

    sigma, width: surface tension and interface thickness D (Eq. 2).
    rho_l, rho_g: densities at phi = +1 and phi = -1 (Eq. 14).
    mobility: M (Eqs. 1, 19).  A: D3Q7 free parameter (Eq. 8).
    s_f: S^f diagonal (Eq. 10).  nu: kinematic viscosity (Eq. 33), which sets
    lambda_9..lambda_13; lambda_g holds the other S^g rates (Eq. 26).
    gravity, rho_ref: body force G = (rho - rho_ref) * gravity.
    stencil: lattice of the finite differences of Eqs. 35-36 (0: D3Q15, the
    default reading; 1: D3Q7).  forcing: 0 uses the printed Eq. 32, 1 the
    untruncated Gamma T of Eq. 28.  lambda_override: nonzero takes
    lambda_9..13 from lambda_g instead of from nu.
    """
    sigma: float = 0.01
    width: float = 4.0
    rho_l: float = 3.0
    rho_g: float = 1.0
    mobility: float = 0.1
    A: float = 0.25
    s_f: Tuple[float, ...] = SF_RT
    nu: float = 0.1
    lambda_g: Tuple[float, ...] = (1.0,) * 15
    gravity: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    rho_ref: float = 0.0
    stencil: int = 0
    forcing: int = 0
    lambda_override: int = 0

    def replace(self, **kw) -> "ModelParams":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Workload:
    name: str
    shape: Tuple[int, int, int]  # (nx, ny, nz)
    bc: Tuple[int, int, int]  # 0 periodic, 1 wall (per axis)
    coupled: bool
    params: ModelParams
    phi0: np.ndarray
    u0: Optional[np.ndarray] = None
    steps: int = 0
    velocity: Optional[dict] = None  # prescribed flow for the interface-tracking runs
    nse_q: int = 15  # lattice of the Navier-Stokes populations: 15 (the paper's) or 19

    @property
    def nodes(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]


def _grid(nx, ny, nz, cell_centred_z=False):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    if cell_centred_z:
        z = z + 0.5
    return x, y, z


def droplet_phi(nx, ny, nz, R, D, centre=None, inside=+1.0):
    """phi = tanh(2 (R - r) / D) around `centre` (default the box centre)."""
    cx, cy, cz = centre if centre is not None else (nx / 2.0, ny / 2.0, nz / 2.0)
    x, y, z = _grid(nx, ny, nz)
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    return inside * np.tanh(2.0 * (R - r) / D)


def rt_phi(W, D, amp=0.05, nx=None, ny=None, nz=None):
    """Rayleigh-Taylor initial field (Eqs. 42-43) on a W x W x 4W box with
    cell-centred z (walls at z = 0 and z = 4W): heavy fluid (phi = +1) on top."""
    nx = W if nx is None else nx
    ny = W if ny is None else ny
    nz = 4 * W if nz is None else nz
    x, y, z = _grid(nx, ny, nz, cell_centred_z=True)
    h = amp * W * (np.cos(2 * np.pi * x / W) + np.cos(2 * np.pi * y / W))
    return np.tanh(2.0 * (z - h - nz / 2.0) / D)


def smooth_field(shape_xyz, rng, amp, modes=3, components=1):
    """Seeded smooth periodic perturbation: a sum of `modes` random low Fourier
    modes per component.  Returns (nz, ny, nx) or (components, nz, ny, nx)."""
    nx, ny, nz = shape_xyz
    x, y, z = _grid(nx, ny, nz)
    out = np.zeros((components, nz, ny, nx))
    for c in range(components):
        for _ in range(modes):
            k = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(-1, 1)
            out[c] += a * np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + ph)
    out *= amp / max(1e-300, np.abs(out).max())
    return out[0] if components == 1 else out


# ---------------------------------------------------------------------------
# The benchmark workloads (lattice sizes and physical numbers of the paper's
# experiments, Sec. III), as concrete parameter records.
# ---------------------------------------------------------------------------

def static_droplet(n=32, R=8.0, D=4.0, sigma=0.01, ratio=3.0, nu=0.1, mobility=0.1, steps=500):
    """Static droplet: n^3 periodic, phi = tanh(2(R - r)/D), rho_l/rho_g = ratio."""
    p = ModelParams(sigma=sigma, width=D, rho_l=ratio, rho_g=1.0, mobility=mobility, s_f=SF_RT, nu=nu)
    return Workload("static_droplet", (n, n, n), (0, 0, 0), True, p, droplet_phi(n, n, n, R, D),
                    steps=steps)


def deformation_flow(n=128, D=3.0, sigma=0.04, U=0.02, T=3.0, Pe=400.0, steps=1000):
    """Interface tracking in the deformation field (Sec. III B, Eq. 41) on an n^3
    periodic box: sphere R = 0.15 n at 0.35 n; mobility from Pe = U R / M."""
    R = 0.15 * n
    c = 0.35 * n
    mob = U * R / Pe
    p = ModelParams(sigma=sigma, width=D, rho_l=1.0, rho_g=1.0, mobility=mob, s_f=SF_ZALESAK, nu=1.0 / 6)
    return Workload("deformation_flow", (n, n, n), (0, 0, 0), False, p,
                    droplet_phi(n, n, n, R, D, centre=(c, c, c)), steps=steps,
                    velocity={"kind": "deformation", "U": U, "T": T})


def zalesak(n=100, R=40.0, slot=16.0, D=2.0, sigma=0.04, U=0.02, Pe=200.0, steps=10000):
    """Zalesak's slotted sphere (Sec. III A, Eq. 37) on an n^3 periodic box,
    centred at n/2, mobility from Pe = U R / M (Eq. 39).  The paper gives the
    slot width only; the slot here is a box of that width along y, cut from
    the bottom of the sphere (-z side) to 2R/3 above the centre (the depth of
    the classic 2D disk, 5R/3).  phi = tanh(2 d / D) with d the signed
    distance of sphere-minus-slot (min/max composition)."""
    c = n / 2.0
    x, y, z = _grid(n, n, n)
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    d_sphere = R - r
    d_outside_slot = np.maximum(np.abs(y - c) - slot / 2.0, z - (c + 2.0 * R / 3.0))
    d = np.minimum(d_sphere, d_outside_slot)
    mob = U * R / Pe
    p = ModelParams(sigma=sigma, width=D, rho_l=1.0, rho_g=1.0, mobility=mob, s_f=SF_ZALESAK, nu=1.0 / 6)
    return Workload("zalesak", (n, n, n), (0, 0, 0), False, p, np.tanh(2.0 * d / D), steps=steps,
                    velocity={"kind": "zalesak", "U": U, "T": 1.0})


def rayleigh_taylor(W=128, Re=1024.0, D=4.0, sigma=1e-4, Pe=50.0, sqrt_gW=0.04, ratio=3.0,
                    steps=1000):
    """Rayleigh-Taylor instability (Sec. III C, Eqs. 42-45): W x W x 4W, periodic
    sides, no-slip top and bottom, Atwood (ratio-1)/(ratio+1), g from sqrt(gW),
    nu from Re = sqrt(gW) W / nu, mobility from Pe = sqrt(gW) W / M."""
    g = sqrt_gW ** 2 / W
    nu = sqrt_gW * W / Re
    mob = sqrt_gW * W / Pe
    p = ModelParams(sigma=sigma, width=D, rho_l=ratio, rho_g=1.0, mobility=mob, s_f=SF_RT, nu=nu,
                    gravity=(0.0, 0.0, -g))
    return Workload(f"rayleigh_taylor_W{W}_Re{int(Re)}", (W, W, 4 * W), (0, 0, 1), True, p,
                    rt_phi(W, D), steps=steps)


def perturbed_case(shape, bc, seed, coupled=True, ratio=3.0, sigma=0.01, D=4.0, nu=0.05,
                   mobility=0.05, gravity=(0.0, 0.0, -2e-5), u_amp=0.02):
    """A droplet off-centre plus seeded smooth perturbations of phi and a seeded
    initial velocity, so that every term of the step is non-zero (parity cases)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    R = 0.3 * min(shape)
    centre = (0.45 * nx, 0.55 * ny, 0.5 * nz)
    phi = droplet_phi(nx, ny, nz, R, D, centre=centre)
    phi = np.clip(phi + smooth_field(shape, rng, 0.05), -1.0, 1.0)
    u0 = smooth_field(shape, rng, u_amp, components=3)
    if bc[2] == 1:  # no flow through the walls at the start
        u0[2][0] = 0.0
        u0[2][-1] = 0.0
    sf = tuple(float(v) for v in (rng.uniform(0.8, 1.6), *([rng.uniform(0.9, 1.5)] * 3),
                                   rng.uniform(0.8, 1.6), rng.uniform(0.8, 1.6), rng.uniform(0.8, 1.6)))
    # S^g: the rates of the conserved-like and energy moments (0, 1, 2) stay
    # near 1 (the paper sets them to 1; far from 1 the scheme is unstable),
    # the others vary over (0.8, 1.6); 9..13 are set from nu anyway
    lam = rng.uniform(0.8, 1.6, size=15)
    lam[0] = rng.uniform(1.0, 1.2)
    lam[1:3] = rng.uniform(0.9, 1.15, size=2)
    lam = tuple(float(v) for v in lam)
    p = ModelParams(sigma=sigma, width=D, rho_l=ratio, rho_g=1.0, mobility=mobility, s_f=sf, nu=nu,
                    lambda_g=lam, gravity=gravity if coupled else (0.0, 0.0, 0.0), rho_ref=0.0)
    return Workload(f"perturbed_{nx}x{ny}x{nz}_s{seed}", shape, bc, coupled, p, phi, u0=u0)


# ---------------------------------------------------------------------------
# Serving trace: independent simulations arriving as a Poisson process.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival: float  # seconds after the trace starts
    kind: str  # "droplet" or "rt"
    shape: Tuple[int, int, int]
    workload: Workload
    steps: int


def serving_trace(n_requests=256, rate_hz=None, steps=2000, seed=20261202, mean_gap_s=0.05,
                  droplet_sizes=(32, 48, 64, 96, 128), rt_widths=(32, 48, 64), rt_steps=None):
    """Seeded trace: half static droplets (box from `droplet_sizes`, R in
    [6, min(20, n/2 - 2D)], density ratio in [1, 10]) and half Rayleigh-Taylor
    boxes W x W x 4W with W from `rt_widths` at Re = 256.  Every request runs
    `steps` steps, the Rayleigh-Taylor ones `rt_steps` if given (at the
    printed parameters a W = 32 box leaves |phi| <= 1 by some 5 % near step
    1000 and fails near step 1800).  Draw order per request: arrival gap,
    kind, size, radius, density ratio."""
    rng = np.random.default_rng(seed)
    gap = mean_gap_s if rate_hz is None else 1.0 / rate_hz
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(rng.exponential(gap))
        kind = "droplet" if rng.uniform() < 0.5 else "rt"
        if kind == "droplet":
            n = int(droplet_sizes[rng.integers(0, len(droplet_sizes))])
            D = 4.0
            rmax = min(20.0, n / 2.0 - 2.0 * D)
            R = float(rng.uniform(6.0, rmax))
            ratio = float(rng.uniform(1.0, 10.0))
            wl = static_droplet(n=n, R=R, D=D, ratio=ratio, steps=steps)
            shape = (n, n, n)
        else:
            W = int(rt_widths[rng.integers(0, len(rt_widths))])
            rng.uniform()  # keep the draw order of the droplet branch
            rng.uniform()
            wl = rayleigh_taylor(W=W, Re=256.0, steps=steps)
            shape = (W, W, 4 * W)
        n_steps = steps if (kind == "droplet" or rt_steps is None) else rt_steps
        out.append(Request(rid, t, kind, shape, wl, n_steps))
    return out


def zero_velocity(shape_xyz):
    nx, ny, nz = shape_xyz
    return np.zeros((3, nz, ny, nx))


def rel_l2(a, b):
    """Relative L2 distance ||a - b|| / max(||b||, 1e-30 sqrt(n))."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.linalg.norm(b)), 1e-30 * math.sqrt(b.size))
    return float(np.linalg.norm(a - b)) / den
