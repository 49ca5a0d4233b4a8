"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the lattice Boltzmann step itself: it
describes workloads (lattice sizes, physical parameters) and generates the
initial macroscopic fields (density and velocity) plus random test states.
Both the GPU library and the oracle turn these fields into populations, each
with its own code.

Initial droplets follow the tanh profile of Eq. (59) between the liquid and
vapour coexistence densities; several droplets combine by taking, at each
node, the droplet whose profile is largest.  The velocity of a droplet is
scaled by its liquid fraction (rho - rho_V) / (rho_L - rho_V).  Coexistence
densities come from ``coexistence.json`` (Maxwell construction, written by
``oracle/make_coexistence.py``), interpolated linearly in T/T_c.
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_COEX = None


def _coex():
    global _COEX
    if _COEX is None:
        with open(os.path.join(HERE, "coexistence.json")) as fh:
            _COEX = json.load(fh)
    return _COEX


def coexistence(T_over_Tc: float) -> tuple[float, float]:
    """(rho_L, rho_V) of the C-S EOS (b=4, R=1) at reduced temperature."""
    rows = np.array(_coex()["carnahan_starling_b4_R1"]["rows"])
    t = float(T_over_Tc)
    if not rows[0, 0] <= t <= rows[-1, 0]:
        raise ValueError(f"T/Tc={t} outside tabulated range")
    return float(np.interp(t, rows[:, 0], rows[:, 1])), float(np.interp(t, rows[:, 0], rows[:, 2]))


def coexistence_exp() -> tuple[float, float]:
    d = _coex()["exponential_G-10/3"]
    return d["rho_L"], d["rho_V"]


# ---------------------------------------------------------------------------
# Physical parameter sets.  Keys are the plain names both sides understand.
# ---------------------------------------------------------------------------
BASE = dict(op="nonorth", psi_form="sqrt_cs", G=-1.0, eos_a=0.5, eos_b=4.0, eos_R=1.0,
            sigma=0.105, tau_nu=1.0, s_e=1.1, s_q=1.2, s_pi=1.4, wall_z=0,
            gravity=(0.0, 0.0, 0.0), theta_wall_deg=90.0, ghost_rho_min=0.0)


def params(nx, ny, nz, **kw) -> dict:
    p = dict(BASE)
    p.update(nx=nx, ny=ny, nz=nz)
    p.update(kw)
    return p


def droplet_fields(nx, ny, nz, droplets, rho_L, rho_V, W, periodic_z=True):
    """Eq. (59) profile for each droplet; returns rho (N,), u (3, N) float64.

    droplets: list of dicts with 'center' (x, y, z), 'r0' and optional 'u'.
    Distances use the minimum image along periodic axes."""
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    z = np.arange(nz, dtype=np.float64)[:, None, None]

    def dist(c, n, periodic):
        d = c
        if periodic:
            d = np.remainder(d + n / 2.0, n) - n / 2.0
        return d

    best = None
    owner = None
    for k, d in enumerate(droplets):
        cx, cy, cz = d["center"]
        dx = dist(x - cx, nx, True)
        dy = dist(y - cy, ny, True)
        dz = dist(z - cz, nz, periodic_z)
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        prof = 0.5 * (rho_L + rho_V) - 0.5 * (rho_L - rho_V) * np.tanh(2.0 * (r - d["r0"]) / W)
        if best is None:
            best = prof
            owner = np.zeros(prof.shape, dtype=np.int64)
        else:
            take = prof > best
            best = np.where(take, prof, best)
            owner = np.where(take, k, owner)
    rho = np.ascontiguousarray(best.reshape(-1))
    u = np.zeros((3, rho.size))
    frac = (rho - rho_V) / (rho_L - rho_V)
    own = owner.reshape(-1)
    for k, d in enumerate(droplets):
        uk = d.get("u", (0.0, 0.0, 0.0))
        m = own == k
        for c in range(3):
            if uk[c] != 0.0:
                u[c, m] = uk[c] * frac[m]
    return rho, u


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def c1_droplet(n=32, T_over_Tc=0.8, r0=8.0, op="nonorth"):
    """Stationary droplet, n^3 periodic, C-S at T/Tc=0.8, radius 8, W=2."""
    p = params(n, n, n, T_over_Tc=T_over_Tc, op=op)
    rl, rv = coexistence(T_over_Tc)
    init = dict(droplets=[dict(center=(n / 2, n / 2, n / 2), r0=r0)], rho_L=rl, rho_V=rv, W=2.0)
    return p, init


def c2_laplace(r0, n=128, op="nonorth"):
    """Laplace-law droplet at 128^3, T/Tc=0.7."""
    p = params(n, n, n, T_over_Tc=0.7, op=op)
    rl, rv = coexistence(0.7)
    init = dict(droplets=[dict(center=(n / 2, n / 2, n / 2), r0=float(r0))], rho_L=rl, rho_V=rv, W=2.0)
    return p, init


def c3_two_droplets(n=256, op="nonorth"):
    """Precision study: 256^3, T/Tc=0.6, a=0.25, two droplets of radius 30
    separated by 70, approaching at 0.05 each, W=5."""
    p = params(n, n, n, T_over_Tc=0.6, eos_a=0.25, op=op)
    rl, rv = coexistence(0.6)
    s = n / 256.0
    c = n / 2.0
    d1 = dict(center=(c - 35.0 * s, c, c), r0=30.0 * s, u=(0.05, 0.0, 0.0))
    d2 = dict(center=(c + 35.0 * s, c, c), r0=30.0 * s, u=(-0.05, 0.0, 0.0))
    init = dict(droplets=[d1, d2], rho_L=rl, rho_V=rv, W=5.0)
    return p, init


def c4_sessile(theta_deg=60.0, nx=384, ny=384, nz=192, r0=40.0):
    """Wall-bounded sessile droplet: periodic x, y; half-way bounce-back walls
    in z; wetting by the Eq. (57) ghost layer; gravity 1e-6 in -z."""
    rl, rv = coexistence(0.7)
    p = params(nx, ny, nz, T_over_Tc=0.7, wall_z=1, theta_wall_deg=float(theta_deg),
               gravity=(0.0, 0.0, -1e-6), ghost_rho_min=0.5 * rv)
    init = dict(droplets=[dict(center=(nx / 2, ny / 2, r0), r0=r0)], rho_L=rl, rho_V=rv, W=2.0,
                periodic_z=False)
    return p, init


def cold_droplet(s_nu, n=16, T_over_Tc=0.5, r0=5.0, storage="f64"):
    """Droplet at T = 0.5 T_c (Maxwell density ratio about 724) with a given
    stress rate s_nu: the large-density-ratio regime where too small a
    viscosity destabilises the scheme (Sec. IV.A)."""
    a, W = interface_recipe(T_over_Tc)
    p = params(n, n, n, T_over_Tc=T_over_Tc, eos_a=a, storage=storage)
    p.pop("tau_nu", None)
    p["s_nu"] = float(s_nu)
    rl, rv = coexistence(T_over_Tc)
    init = dict(droplets=[dict(center=(n / 2, n / 2, n / 2), r0=r0)], rho_L=rl, rho_V=rv, W=W)
    return p, init


def interface_recipe(T_over_Tc):
    """EOS constant a and initial interface width W for a reduced temperature:
    linear between the paper's T = 0.6 T_c setting (a = 0.25, W = 5, about
    five lattice units of interface) and a = 0.5, W = 2 at T = 0.9 T_c.  With
    a = 0.5 and W = 2 a droplet at T = 0.6 T_c diverges within a few steps
    (checked with the oracle)."""
    s = (float(T_over_Tc) - 0.6) / 0.3
    return 0.25 + 0.25 * s, 5.0 - 3.0 * s


def c5_batch(n_runs=256, seed=1805, sizes=(32, 48, 64, 96)):
    """Independent periodic droplet runs: L ~ U{sizes}, r0 = L/4 + U[-2, 2],
    T/Tc ~ U[0.6, 0.9], tau_nu ~ U[0.6, 1.2]; drawn per run in that order.
    a and W follow ``interface_recipe``."""
    rng = np.random.default_rng(seed)
    runs = []
    for _ in range(n_runs):
        L = int(rng.choice(sizes))
        dr = float(rng.uniform(-2.0, 2.0))
        t = float(rng.uniform(0.6, 0.9))
        tau = float(rng.uniform(0.6, 1.2))
        a, W = interface_recipe(t)
        p = params(L, L, L, T_over_Tc=t, tau_nu=tau, eos_a=a)
        rl, rv = coexistence(t)
        init = dict(droplets=[dict(center=(L / 2, L / 2, L / 2), r0=0.25 * L + dr)],
                    rho_L=rl, rho_V=rv, W=W)
        runs.append((p, init))
    return runs


def init_fields(p, init):
    """rho (N,), u (3, N) for a workload's initial condition."""
    return droplet_fields(p["nx"], p["ny"], p["nz"], init["droplets"], init["rho_L"],
                          init["rho_V"], init["W"], periodic_z=init.get("periodic_z", True))


def random_fields(nx, ny, nz, seed, rho_lo=0.05, rho_hi=0.35, umax=0.05):
    """Smooth-free random density/velocity fields (uniform), for unit tests."""
    rng = np.random.default_rng(seed)
    N = nx * ny * nz
    rho = rng.uniform(rho_lo, rho_hi, N)
    u = rng.uniform(-umax, umax, (3, N))
    return rho, u


def random_populations(nx, ny, nz, seed, lo=0.002, hi=0.02):
    """Random positive populations (19, N), for operator tests."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (19, nx * ny * nz))
