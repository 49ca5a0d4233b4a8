"""ctypes glue between Python and the C oracle (test infrastructure).

``make_params`` turns a plain parameter dict (the workload description) into
the C struct, attaching the exact matrices from ``oracle.moments``.
Parameter mapping, all from the paper:
  * s_nu = 1 / tau_nu (Eq. (54) then gives nu = c_s^2 (tau_nu - 1/2));
  * T = (T/T_c) * 0.37733 a / (b R)  (text after Eq. (58));
  * tan_wall = tan(90 deg - theta_a)  (Eq. (57)).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import moments
from .build import LIB, build

Q = 19


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("wall_z", ctypes.c_int32), ("op", ctypes.c_int32), ("psi_form", ctypes.c_int32),
        ("nthreads", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("G", ctypes.c_double),
        ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double), ("eos_R", ctypes.c_double),
        ("eos_T", ctypes.c_double),
        ("psi0", ctypes.c_double), ("rho0", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("tan_wall", ctypes.c_double),
        ("ghost_rho_min", ctypes.c_double),
        ("orth_sig_e", ctypes.c_double), ("orth_sig_eps", ctypes.c_double),
        ("rates", ctypes.c_double * Q),
        ("M", ctypes.c_double * (Q * Q)),
        ("Minv", ctypes.c_double * (Q * Q)),
        ("nu_mask", ctypes.c_int32), ("reserved2", ctypes.c_int32),
        ("nu_ratio", ctypes.c_double), ("visc_rho_L", ctypes.c_double), ("visc_rho_V", ctypes.c_double),
        ("wall_x", ctypes.c_int32), ("wall_y", ctypes.c_int32),
        ("lid_u", ctypes.c_double * 3), ("lid_rho", ctypes.c_double),
        ("orth_meq", ctypes.c_int32), ("reserved3", ctypes.c_int32),
    ]


_lib = None


def load(path: str):
    """Open an oracle library (the default one, or a variant the tests
    built) and declare its entry points."""
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(OracleParams)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    L.oracle_step.argtypes = [P, dp, dp, i64]
    L.oracle_collide_nodes.argtypes = [P, dp, i64, ctypes.POINTER(ctypes.c_int64), dp]
    L.oracle_equilibrium.argtypes = [P, dp, dp, dp]
    L.oracle_fields.argtypes = [P, dp, dp, dp, dp, dp, dp]
    L.oracle_psi_array.argtypes = [P, dp, dp, i64]
    for fn in ("oracle_step", "oracle_collide_nodes", "oracle_equilibrium",
               "oracle_fields", "oracle_psi_array"):
        getattr(L, fn).restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = load(LIB if os.path.exists(LIB) else build())
    return _lib


_MATS = {}


def _matrices(op: str):
    if op not in _MATS:
        if op == "nonorth":
            M = moments.nonorth_M()
        elif op == "orth":
            M = moments.orth_M()
        else:
            raise ValueError(op)
        _MATS[op] = (moments.to_f64(M), moments.to_f64(moments.exact_inverse(M)))
    return _MATS[op]


def temperature(cfg) -> float:
    """Absolute T from T/T_c with T_c = 0.37733 a / (b R)."""
    return cfg["T_over_Tc"] * 0.37733 * cfg["eos_a"] / (cfg["eos_b"] * cfg["eos_R"])


def rates_of(cfg):
    if "rates" in cfg:
        return list(cfg["rates"])
    s_nu = 1.0 / cfg["tau_nu"] if "tau_nu" in cfg else cfg["s_nu"]
    if cfg.get("op", "nonorth") == "nonorth":
        return moments.nonorth_rates(cfg["s_e"], s_nu, cfg["s_q"], cfg["s_pi"])
    return moments.orth_rates(cfg["s_e"], s_nu, cfg["s_q"], cfg["s_pi"],
                              cfg.get("s_eps", cfg["s_pi"]), cfg.get("s_m", cfg["s_q"]))


def make_params(cfg: dict, nthreads: int = 0) -> OracleParams:
    p = OracleParams()
    p.nx, p.ny, p.nz = cfg["nx"], cfg["ny"], cfg["nz"]
    p.wall_z = int(cfg.get("wall_z", 0))
    op = cfg.get("op", "nonorth")
    p.op = {"nonorth": 0, "orth": 1}[op]
    p.psi_form = {"sqrt_cs": 0, "exp": 1}[cfg.get("psi_form", "sqrt_cs")]
    p.nthreads = nthreads
    p.G = cfg["G"]
    p.eos_a = cfg.get("eos_a", 0.5)
    p.eos_b = cfg.get("eos_b", 4.0)
    p.eos_R = cfg.get("eos_R", 1.0)
    p.eos_T = temperature({**cfg, "eos_a": p.eos_a, "eos_b": p.eos_b, "eos_R": p.eos_R,
                           "T_over_Tc": cfg.get("T_over_Tc", 0.0)})
    p.psi0 = cfg.get("psi0", 1.0)
    p.rho0 = cfg.get("rho0", 1.0)
    p.sigma = cfg.get("sigma", 0.0)
    g = cfg.get("gravity", (0.0, 0.0, 0.0))
    for d in range(3):
        p.g[d] = g[d]
    p.tan_wall = math.tan(math.radians(90.0 - cfg.get("theta_wall_deg", 90.0)))
    p.ghost_rho_min = cfg.get("ghost_rho_min", 0.0)
    ce, ceps = moments.orth_sigma_rows()
    p.orth_sig_e, p.orth_sig_eps = float(ce), float(ceps)
    # Readings of the orthogonal model: the Eq. (16) term on the e row only
    # (orth_sigma = 0, the default) or also on the eps row (1); the
    # alternative equilibrium of the eps and pi rows (orth_meq = 1).
    if not int(cfg.get("orth_sigma", 0)):
        p.orth_sig_eps = 0.0
    p.orth_meq = int(cfg.get("orth_meq", 0))
    r = rates_of(cfg)
    for k in range(Q):
        p.rates[k] = r[k]
    M, Mi = _matrices(op)
    ctypes.memmove(p.M, M.ctypes.data, M.nbytes)
    ctypes.memmove(p.Minv, Mi.ctypes.data, Mi.nbytes)
    rows = moments.NONORTH_NU_ROWS if op == "nonorth" else moments.orth_nu_rows()
    p.nu_mask = sum(1 << k for k in rows)
    p.nu_ratio = float(cfg.get("nu_ratio", 0.0))
    p.visc_rho_L = float(cfg.get("visc_rho_L", 0.0))
    p.visc_rho_V = float(cfg.get("visc_rho_V", 0.0))
    p.wall_x = int(cfg.get("wall_x", 0))
    p.wall_y = int(cfg.get("wall_y", 0))
    lu = cfg.get("lid_u", (0.0, 0.0, 0.0))
    for d in range(3):
        p.lid_u[d] = float(lu[d])
    p.lid_rho = float(cfg.get("lid_rho", 1.0))
    return p


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, fn):
    if rc != 0:
        raise RuntimeError(f"{fn} failed with code {rc}")


def nnodes(p):
    return p.nx * p.ny * p.nz


def equilibrium(p: OracleParams, rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """fbar(x) = M^-1 m_eq(rho(x), u(x)); rho shape (N,), u shape (3, N)."""
    N = nnodes(p)
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(N)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, N)
    f = np.empty((Q, N))
    _check(lib().oracle_equilibrium(ctypes.byref(p), _dp(rho), _dp(u), _dp(f)), "equilibrium")
    return f


def step(p: OracleParams, f: np.ndarray, nsteps: int = 1) -> np.ndarray:
    N = nnodes(p)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q, N)
    out = np.empty_like(f)
    _check(lib().oracle_step(ctypes.byref(p), _dp(f), _dp(out), nsteps), "step")
    return out


def collide_nodes(p: OracleParams, f: np.ndarray, idx) -> np.ndarray:
    """Post-collision fbar*(x, t) at node indices idx (shape (n, 19))."""
    N = nnodes(p)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q, N)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((len(idx), Q))
    _check(lib().oracle_collide_nodes(ctypes.byref(p), _dp(f), len(idx),
                                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      _dp(out)), "collide_nodes")
    return out


def step_sampled(p: OracleParams, f: np.ndarray, idx) -> np.ndarray:
    """fbar(x, t+1) at the nodes idx, one node at a time: each direction a pulls
    fbar*_a from x - e_a (Eq. (5)), or bounces fbar*_opp(a) back at x when
    x - e_a lies beyond a wall.  Returns shape (n, 19)."""
    nx, ny, nz = p.nx, p.ny, p.nz
    idx = np.asarray(idx, dtype=np.int64)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    src_nodes, src_dir = [], []
    for a, (ex, ey, ez) in enumerate(moments.VELOCITIES):
        sz = z - ez
        if p.wall_z:
            out = (sz < 0) | (sz >= nz)
        else:
            out = np.zeros_like(sz, dtype=bool)
        sx, sy, szw = (x - ex) % nx, (y - ey) % ny, sz % nz
        src = np.where(out, idx, (szw * ny + sy) * nx + sx)
        d = np.where(out, moments.opposite(a), a)
        src_nodes.append(src)
        src_dir.append(d)
    src_nodes = np.stack(src_nodes, axis=1)  # (n, 19)
    src_dir = np.stack(src_dir, axis=1)
    uniq, inv = np.unique(src_nodes.reshape(-1), return_inverse=True)
    post = collide_nodes(p, f, uniq)  # (u, 19)
    inv = inv.reshape(src_nodes.shape)
    return post[inv, src_dir]


def fields(p: OracleParams, f: np.ndarray, L=None) -> dict:
    """rho, u, total force F, psi and p of the state f (L: an oracle library
    from ``load``; default the built one)."""
    N = nnodes(p)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q, N)
    rho, psi, pr = np.empty(N), np.empty(N), np.empty(N)
    u, F = np.empty((3, N)), np.empty((3, N))
    _check((L or lib()).oracle_fields(ctypes.byref(p), _dp(f), _dp(rho), _dp(u), _dp(F),
                               _dp(psi), _dp(pr)), "fields")
    return {"rho": rho, "u": u, "F": F, "psi": psi, "p": pr}


def psi(p: OracleParams, rho) -> np.ndarray:
    rho = np.ascontiguousarray(np.atleast_1d(rho), dtype=np.float64)
    out = np.empty_like(rho)
    _check(lib().oracle_psi_array(ctypes.byref(p), _dp(rho), _dp(out), len(rho)), "psi")
    return out


def pressure_fn(p: OracleParams):
    """p(rho) = rho c_s^2 + G psi(rho)^2 / 2 using the C oracle's psi."""
    def pr(r):
        ps = psi(p, r)[0]
        return r / 3.0 + 0.5 * p.G * ps * ps
    return pr
