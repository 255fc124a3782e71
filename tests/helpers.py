"""Shared test helpers: run a workload through the oracle or the GPU library,
compare fields, and evaluate the oracle on a window around sampled nodes."""
from __future__ import annotations

import numpy as np

import oracle.orc as orc
from paper_1507_07294_amd import workloads as wl

FIELDS = ("phi", "rho", "mu", "ux", "uy", "uz", "p")


def oracle_for(w):
    mode = (orc.COUPLED_Q19 if w.nse_q == 19 else orc.COUPLED) if w.coupled else orc.CHE_ONLY
    o = orc.Oracle(w.shape, w.bc, mode, w.params)
    if not w.coupled:
        v = w.velocity or {"kind": "zero"}
        kind = {"zero": orc.VEL_ZERO, "field": orc.VEL_FIELD, "zalesak": orc.VEL_ZALESAK,
                "deformation": orc.VEL_DEFORM}[v["kind"]]
        o.set_velocity(kind, v.get("field"), v.get("U", 0.0), v.get("T", 1.0))
    o.init(w.phi0, w.u0 if w.coupled else None)
    return o


def gpu_for(w, precision="f64"):
    from paper_1507_07294_amd import mplb
    return mplb.from_workload(w, precision)


def fields_of(sim, coupled=True):
    keys = FIELDS if coupled else ("phi", "rho", "mu", "ux", "uy", "uz")
    return {k: sim.read(k) for k in keys}


# Floors of the relative L2 metric, in lattice units (c = 1): fields whose
# RMS falls below these (a pressure that is 0 up to O(u^2), a chemical
# potential in the bulk) are compared on this absolute scale instead.  The
# pressure floor is the scale of sigma/R and rho u^2 in the test cases:
# Eq. 30 forms p from O(rho |u|) populations, so its round-off is set by
# them, not by p itself.
FLOORS = {"phi": 1e-6, "rho": 1e-6, "mu": 1e-8, "ux": 1e-6, "uy": 1e-6, "uz": 1e-6, "p": 1e-5}


def rel_err(a, b, floor=0.0):
    """||a - b|| / max(||b||, floor sqrt(n))."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.linalg.norm(b)), floor * np.sqrt(b.size), 1e-300)
    return float(np.linalg.norm(a - b)) / den


def rel_errors(a, b):
    return {k: rel_err(a[k], b[k], FLOORS.get(k, 0.0)) for k in b}


def mu_error_bound(params, dphi_rms, eps):
    """Bound on the RMS error of mu = 4 beta (phi^3 - phi) - kappa lap phi
    (Eqs. 2, 36) that a phi error of RMS dphi_rms, plus rounding at unit
    round-off eps in the evaluation itself, can cause.  The double-well term
    has slope 4 beta (3 phi^2 - 1) <= 8 beta for |phi| <= 1; the isotropic
    Laplacian's stencil (weights 2 w_i / c_s^2) has an absolute coefficient
    sum 12 (1 - w_0) <= 12, which bounds its L2 gain (Young's inequality).
    The bound holds at any lattice size, where the relative L2 of mu does not:
    mu vanishes in the bulk, so its norm grows with the interface area while
    the round-off grows with the volume."""
    beta = 3.0 * params.sigma / (4.0 * params.width)
    kappa = 3.0 * params.width * params.sigma / 8.0
    return (8.0 * beta + 12.0 * kappa) * dphi_rms + eps * (12.0 * beta + 12.0 * kappa)


# ---------------------------------------------------------------------------
# Windowed oracle: fields at sampled nodes of a lattice too large for the
# oracle.  After n steps a node depends on the initial state within 3 hops
# per step plus 3 for the read-out (pull 1, finite differences 2), so a
# window of radius r >= 3n + 3 reproduces it exactly; outside periodic axes
# the window wraps onto itself, which only corrupts nodes more than r away.
# ---------------------------------------------------------------------------

def _axis_window(c, n, r, wall):
    if 2 * r + 1 >= n:
        return np.arange(n), True, c  # whole axis, its own boundary condition
    if wall:
        lo, hi = max(0, c - r), min(n - 1, c + r)
        return np.arange(lo, hi + 1), False, c - lo
    return (np.arange(c - r, c + r + 1) % n), False, r


def window_oracle_fields(w, node_xyz, steps):
    """Oracle fields at `node_xyz` after `steps` steps, computed on a window
    (coupled lattices, and CHE-only lattices at rest: the step is then the same
    at every node, while a prescribed flow depends on absolute position)."""
    assert w.coupled or (w.velocity or {"kind": "zero"})["kind"] == "zero"
    r = 3 * steps + 4
    nx, ny, nz = w.shape
    x, y, z = node_xyz
    ix, fx, cx = _axis_window(x, nx, r, w.bc[0] == 1)
    iy, fy, cy = _axis_window(y, ny, r, w.bc[1] == 1)
    iz, fz, cz = _axis_window(z, nz, r, w.bc[2] == 1)
    sub = np.ix_(iz, iy, ix)
    phi = w.phi0[sub]
    u0 = None if w.u0 is None else np.stack([w.u0[a][sub] for a in range(3)])
    # every axis keeps its boundary condition: walls stay walls (a clipped
    # window edge that is not the real wall lies more than r away), periodic
    # axes wrap (onto themselves when the window is narrower than the axis)
    bc = tuple(w.bc)
    sw = wl.Workload(w.name + "_window", (len(ix), len(iy), len(iz)), bc, w.coupled, w.params, phi, u0=u0,
                     velocity=w.velocity, nse_q=w.nse_q)
    o = oracle_for(sw)
    o.step(steps)
    return {k: float(o.read(k)[cz, cy, cx]) for k in (FIELDS if w.coupled else ("phi", "mu"))}
