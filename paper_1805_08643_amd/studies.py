"""Physics studies on the GPU path, compared with what the paper reports.

Each study advances lattices with the HIP library through the binding and
returns plain dicts (one line of JSON per run is printed as it finishes).

  table1     Sec. IV.A, Table I: phase separation with psi = exp(-1/rho),
             G = -10/3, 120^3, rho = 1 - U[0, 10]/5000, s_e = 0.8, other
             non-conserved rates 1.2, nu in {0.01, 0.05, 0.1, 0.15}, both
             operators, 8000 steps; bulk liquid / vapour densities.
  stability  Sec. IV.A: the same run at nu = 1e-3 (the paper: diverges) and
             nu = 2e-3 (the paper: stable).
  laplace    Sec. IV.B, Fig. 2: static droplets, exponential psi, 150^3,
             nu = 0.1; Delta p against 1 / R_d, linear fit.
  spurious   Sec. IV.B, Fig. 3: maximum spurious velocity, exponential psi,
             80^3, r0 = 15, 1/s_nu from 0.55 to 1.0, both operators.
  contact    Sec. IV.C: sessile droplet with the Eq. (57) ghost layer,
             exponential psi, 160 x 160 x 120, r0 = 30, nu = 0.1, prescribed
             angles 30, 60, 90, 135 deg.
  flat       Sec. IV.D, Fig. 5: flat interfaces at z = 0.25 N_z and 0.75 N_z,
             C-S EOS with a = 0.5, sigma = 0.116, 1/s_nu = 0.8, 100^3;
             coexistence densities against the Maxwell construction.
  table2     Sec. IV.D, Table II and Fig. 6: droplet at T = 0.6 T_c, a = 0.25,
             120^3, r0 = 40, W = 5, sigma = 0.105, both operators;
             coexistence densities and maximum spurious velocity.
  viscosity_ratio  Sec. IV.D after Fig. 6: the same droplet with nu_L = 0.01
             and nu_V / nu_L in {1, 2, 5, 10}; maximum spurious velocity.
  cavity_cost  Appendix B, Table III: time of 5000 iterations of the
             single-phase lid-driven cavity, L = 60, 80, 110, both operators.
  laplace_cs Laplace law with the C-S EOS at T = 0.7 T_c, a = 0.5, 128^3,
             r0 in 12..28, FP64 and FP32 storage, both operators.
  contact_cs Sessile droplet with the C-S EOS at T = 0.7 T_c on
             384 x 384 x 192, gravity 1e-6 along -z, 60 / 90 / 120 deg, FP32.
  contact_precision  the same wall-bounded configuration with gravity in
             FP64, FP32 and F16N storage: contact angle, density field and
             spurious currents against FP64 storage.
  storage_drift  mass drift of each storage format over 50,000 steps of a
             96 x 96 x 48 sessile droplet, with and without gravity.
  throughput GPU MLUPS for each standard workload.
  precision  FP32 and 16-bit storage (F16S with three shifts, F16N) against
             FP64 storage on the 256^3 two-droplet run (steps 100, 500, 1000,
             2000).
  precision_results  per-result errors of FP32, F16S and F16N storage against
             FP64 storage on the 128^3 Laplace droplets at rest: coexistence
             densities, Delta p, surface tension, spurious currents, density
             field.

``python -m paper_1805_08643_amd.studies <name> [<name> ...] [--out-dir DIR]``
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

# Rates of the paper-replication runs (Sec. IV.A): s_e = 0.8, the other
# non-conserved rates 1.2, s_nu from the viscosity.
PAPER_RATES = dict(s_e=0.8, s_q=1.2, s_pi=1.2, s_eps=1.2, s_m=1.2)
# Exponential pseudopotential of Secs. IV.A-C.
EXP_PSI = dict(psi_form="exp", G=-10.0 / 3.0, psi0=1.0, rho0=1.0, sigma=0.0)


def tau_for_nu(nu):
    """1 / s_nu from the kinematic viscosity, Eq. (54): nu = (1/s_nu - 1/2) / 3."""
    return 3.0 * nu + 0.5


def _emit(rec):
    print(json.dumps(rec), flush=True)
    return rec


def _bulk(rho, frac=0.01):
    """Plateau densities: means of the nodes within frac of the range from
    the maximum (liquid) and from the minimum (vapour)."""
    lo, hi = float(rho.min()), float(rho.max())
    band = frac * (hi - lo)
    return float(rho[rho >= hi - band].mean()), float(rho[rho <= lo + band].mean())


def _droplet(lat, center, R, W):
    """Mean density and pressure inside r < R/2 and outside r > R + 2W, the
    equal-volume radius from the total mass, and max |u|."""
    d = lat.diagnostics(center=center, r_in=0.5 * R, r_out=R + 2.0 * W)
    rl = d["rho_in"] / d["n_in"]
    rv = d["rho_out"] / d["n_out"]
    dp = d["p_in"] / d["n_in"] - d["p_out"] / d["n_out"]
    Rd = (3.0 * (d["mass"] - rv * lat.N) / (4.0 * math.pi * (rl - rv))) ** (1.0 / 3.0)
    return dict(rho_L=rl, rho_V=rv, dp=dp, R_d=Rd, max_u=d["max_u"], mass=d["mass"], nonfinite=d["nonfinite"])


def _linfit(x, y):
    A = np.vstack([x, np.ones_like(x)]).T
    (slope, icpt), *_ = np.linalg.lstsq(A, y, rcond=None)
    pred = A @ np.array([slope, icpt])
    r2 = 1.0 - ((y - pred) ** 2).sum() / ((y - y.mean()) ** 2).sum()
    return float(slope), float(icpt), float(r2)


def _lattice(cfg):
    from paper_1805_08643_amd.binding import Lattice
    return Lattice(cfg)


def _params(n, **kw):
    import lbm_inputs as li
    return li.params(*(n if isinstance(n, tuple) else (n, n, n)), **kw)


# --------------------------------------------------------------------------
# Sec. IV.A
# --------------------------------------------------------------------------
def _phase_separation(nu, op, n, seed, storage):
    cfg = _params(n, op=op, tau_nu=tau_for_nu(nu), storage=storage, **EXP_PSI, **PAPER_RATES)
    return _phase_separation_cfg(cfg, seed)


def _phase_separation_cfg(cfg, seed):
    n3 = cfg["nx"] * cfg["ny"] * cfg["nz"]
    rng = np.random.default_rng(seed)
    rho = 1.0 - rng.uniform(0.0, 10.0, n3) / 5000.0
    lat = _lattice(cfg)
    lat.init_fields(rho, np.zeros((3, n3)))
    return lat


def table1(ops=("nonorth", "orth"), nus=(0.01, 0.05, 0.1, 0.15), steps=8000, n=120, seed=1805, storage="f64"):
    out = []
    for op in ops:
        for nu in nus:
            t0 = time.time()
            lat = _phase_separation(nu, op, n, seed, storage)
            lat.step(steps)
            rho = lat.read_fields()["rho"].cpu().numpy()
            d = lat.diagnostics()
            lat.close()
            rl, rv = _bulk(rho)
            out.append(_emit(dict(study="table1", op=op, nu=nu, steps=steps, rho_L=rl, rho_V=rv,
                                  max_u=d["max_u"], nonfinite=d["nonfinite"], seconds=round(time.time() - t0, 1))))
    return out


def stability(nus=(1e-3, 2e-3), ops=("nonorth", "orth"), steps=8000, n=120, seed=1805, chunk=250):
    out = []
    for op in ops:
        for nu in nus:
            lat = _phase_separation(nu, op, n, seed, "f64")
            diverged = None
            for k in range(steps // chunk):
                lat.step(chunk)
                d = lat.diagnostics()
                if d["nonfinite"] or not math.isfinite(d["max_u"]) or d["max_u"] > 0.5:
                    diverged = (k + 1) * chunk
                    break
            lat.close()
            out.append(_emit(dict(study="stability", op=op, nu=nu, steps=steps, diverged_by_step=diverged,
                                  max_u=d["max_u"])))
    return out


# --------------------------------------------------------------------------
# Sec. IV.B
# --------------------------------------------------------------------------
def _exp_droplet(n, r0, nu, op, storage, W=4.0):
    import lbm_inputs as li
    rl, rv = li.coexistence_exp()
    cfg = _params(n, op=op, tau_nu=tau_for_nu(nu), storage=storage, **EXP_PSI, **PAPER_RATES)
    c = (n / 2, n / 2, n / 2)
    lat = _lattice(cfg)
    lat.init_droplets([dict(center=c, r0=float(r0))], rl, rv, W)
    return lat, c


def laplace(ops=("nonorth", "orth"), radii=(20, 25, 30, 35, 40), steps=20000, n=150, storage="f64"):
    """Radii from 20: at r0 = 15 in a 150^3 box the droplet evaporates, the
    vapour initialised at the flat-interface density being below the
    higher vapour density a small droplet needs (Kelvin effect)."""
    out = {}
    for op in ops:
        pts = []
        for r0 in radii:
            lat, c = _exp_droplet(n, r0, 0.1, op, storage)
            lat.step(steps)
            pts.append(_emit(dict(study="laplace", op=op, r0=r0, **_droplet(lat, c, r0, 4.0))))
            lat.close()
        x = np.array([1.0 / p["R_d"] for p in pts])
        y = np.array([p["dp"] for p in pts])
        slope, icpt, r2 = _linfit(x, y)
        out[op] = _emit(dict(study="laplace_fit", op=op, slope=slope, surface_tension=slope / 2, intercept=icpt,
                             r2=r2, max_dp=float(y.max()), steps=steps, n=n, points=pts))
    return out


def spurious(ops=("nonorth", "orth"), inv_s_nu=(0.55, 0.6, 0.7, 0.8, 0.9, 1.0), steps=20000, n=80, r0=15.0):
    out = []
    for op in ops:
        for t in inv_s_nu:
            lat, c = _exp_droplet(n, r0, (t - 0.5) / 3.0, op, "f64")
            lat.step(steps)
            out.append(_emit(dict(study="spurious", op=op, inv_s_nu=t, steps=steps, **_droplet(lat, c, r0, 4.0))))
            lat.close()
    return out


# --------------------------------------------------------------------------
# Sec. IV.C
# --------------------------------------------------------------------------
def contact_angle(rho, nx, ny, nz, rho_mid, zmin=3, zw=0.0):
    """Angle through the liquid where the droplet meets the plane z = zw,
    from a sphere fitted (algebraic least squares) to the rho = rho_mid
    isosurface above z = zmin; crossings found by linear interpolation along
    x, y and z.  Also returns the cap formula 2 atan(h / r_b) with h the
    apex height above that plane and r_b the base radius there.

    Eq. (57) prescribes the angle through a central difference about the
    first fluid layer (z = 0), so zw = 0 is the plane it acts on; the
    half-way bounce-back wall itself sits at z = -1/2."""
    a = rho.reshape(nz, ny, nx)
    pts = []
    for axis in range(3):
        n = a.shape[axis]
        lo = np.take(a, np.arange(n - 1), axis=axis)
        hi = np.take(a, np.arange(1, n), axis=axis)
        cross = (lo - rho_mid) * (hi - rho_mid) < 0
        idx = np.argwhere(cross).astype(np.float64)
        if len(idx) == 0:
            continue
        t = (rho_mid - lo[cross]) / (hi[cross] - lo[cross])
        idx[:, axis] += t
        pts.append(idx)
    P = np.concatenate(pts)[:, ::-1]  # x, y, z
    P = P[P[:, 2] >= zmin]
    A = np.hstack([2.0 * P, np.ones((len(P), 1))])
    sol, *_ = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)
    c = sol[:3]
    R = math.sqrt(sol[3] + (c ** 2).sum())
    theta = math.degrees(math.acos(max(-1.0, min(1.0, (zw - c[2]) / R))))
    h = c[2] + R - zw
    rb2 = R * R - (c[2] - zw) ** 2
    cap = math.degrees(2.0 * math.atan2(h, math.sqrt(rb2))) if rb2 > 0 else float("nan")
    return theta, dict(center=[float(v) for v in c], radius=R, points=int(len(P)), cap_formula_deg=cap)


def _sessile(cfg, droplet, rl, rv, W, steps, storage):
    cfg = dict(cfg, storage=storage)
    lat = _lattice(cfg)
    lat.init_droplets([droplet], rl, rv, W)
    lat.step(steps)
    rho = lat.read_fields()["rho"].cpu().numpy()
    d = lat.diagnostics()
    lat.close()
    mid = 0.5 * (rl + rv)
    th, fit = contact_angle(rho, cfg["nx"], cfg["ny"], cfg["nz"], mid)
    fit["theta_at_bounce_back_plane"] = contact_angle(rho, cfg["nx"], cfg["ny"], cfg["nz"], mid, zw=-0.5)[0]
    return th, fit, d


def contact(thetas=(30.0, 60.0, 90.0, 135.0), steps=40000, nx=160, ny=160, nz=120, r0=30.0, storage="f64"):
    import lbm_inputs as li
    rl, rv = li.coexistence_exp()
    out = []
    for th in thetas:
        t0 = time.time()
        cfg = _params((nx, ny, nz), tau_nu=tau_for_nu(0.1), wall_z=1, theta_wall_deg=th, ghost_rho_min=0.5 * rv,
                      **EXP_PSI, **PAPER_RATES)
        drop = dict(center=(nx / 2, ny / 2, r0), r0=r0)
        ang, fit, d = _sessile(cfg, drop, rl, rv, 4.0, steps, storage)
        out.append(_emit(dict(study="contact", theta_prescribed=th, theta_measured=ang, fit=fit, steps=steps,
                              max_u=d["max_u"], mass=d["mass"], seconds=round(time.time() - t0, 1))))
    return out


def contact_cs(thetas=(60.0, 90.0, 120.0), steps=50000, storage="f32", gravity=(True, False)):
    """With the config's gravity (1e-6 along -z; Bond number about 0.1, so the
    droplet is flattened and a sphere fit reads low) and without it."""
    import lbm_inputs as li
    out = []
    for th, gr in [(t, g) for g in gravity for t in thetas]:
        t0 = time.time()
        cfg, init = li.c4_sessile(th)
        if not gr:
            cfg = dict(cfg, gravity=(0.0, 0.0, 0.0))
        ang, fit, d = _sessile(cfg, init["droplets"][0], init["rho_L"], init["rho_V"], init["W"], steps, storage)
        out.append(_emit(dict(study="contact_cs", theta_prescribed=th, theta_measured=ang, fit=fit, steps=steps,
                              storage=storage, gravity=list(cfg["gravity"]), max_u=d["max_u"], mass=d["mass"], seconds=round(time.time() - t0, 1))))
    return out


def contact_precision(thetas=(60.0, 90.0, 120.0), steps=50000, storages=("f64", "f32", "f16n")):
    """The wall-bounded configuration (384 x 384 x 192 sessile droplet, C-S
    EOS at T = 0.7 T_c, gravity 1e-6 along -z, Eq. (57) wetting layer) in
    each storage format for `steps` steps: the measured contact angle, the
    density field and the spurious currents of FP32 and F16N against the same
    run in FP64 storage."""
    import torch

    import lbm_inputs as li
    from paper_1805_08643_amd.binding import f16_exp_for
    out = []
    for th in thetas:
        cfg, init = li.c4_sessile(th)
        rl, rv = init["rho_L"], init["rho_V"]
        ref = None
        for st in storages:
            t0 = time.time()
            c = dict(cfg, storage=st, rho_ref=rv, f16_exp=f16_exp_for(1.25 * rl))
            lat = _lattice(c)
            lat.init_droplets(init["droplets"], rl, rv, init["W"])
            m0 = lat.diagnostics()["mass"]
            lat.step(steps)
            rho = lat.read_fields()["rho"].cpu().numpy()
            d = lat.diagnostics()
            lat.close()
            torch.cuda.empty_cache()
            ang, fit = contact_angle(rho, cfg["nx"], cfg["ny"], cfg["nz"], 0.5 * (rl + rv))
            row = dict(study="contact_precision", theta_prescribed=th, storage=st, steps=steps, theta_measured=ang,
                       max_u=d["max_u"], mass_drift=(d["mass"] - m0) / m0, seconds=round(time.time() - t0, 1))
            if ref is None:
                ref = (rho, ang, d["max_u"])
            else:
                rel = np.abs(rho - ref[0]) / ref[0]
                liquid = ref[0] > 0.5 * (rl + rv)
                row.update(theta_err_deg=ang - ref[1], max_u_rel_err=abs(d["max_u"] - ref[2]) / ref[2],
                           rho_max_rel_err_liquid=float(rel[liquid].max()),
                           rho_max_rel_err_vapour=float(rel[~liquid].max()))
            out.append(_emit(row))
        del ref
    return out


def storage_drift(n=96, nz=48, r0=12.0, theta=60.0, steps=50000, every=5000,
                  storages=("f64", "f32", "f16s", "f16n"), gravity=(True, False)):
    """Relative mass drift over a long run of a small sessile droplet (the
    wall-bounded configuration scaled to n x n x nz) in each storage format,
    every `every` steps, with and without gravity."""
    import lbm_inputs as li
    from paper_1805_08643_amd.binding import f16_exp_for
    out = []
    for gr in gravity:
        cfg, init = li.c4_sessile(theta, nx=n, ny=n, nz=nz, r0=r0)
        if not gr:
            cfg = dict(cfg, gravity=(0.0, 0.0, 0.0))
        for st in storages:
            c = dict(cfg, storage=st, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
            lat = _lattice(c)
            lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
            m0 = lat.diagnostics()["mass"]
            drift = []
            for _ in range(steps // every):
                lat.step(every)
                drift.append((lat.diagnostics()["mass"] - m0) / m0)
            lat.close()
            out.append(_emit(dict(study="storage_drift", storage=st, gravity=list(cfg["gravity"]), size=[n, n, nz],
                                  theta=theta, every=every, mass_drift=drift)))
    return out


# --------------------------------------------------------------------------
# Sec. IV.D
# --------------------------------------------------------------------------
def flat(temps=(0.6, 0.65, 0.7, 0.75, 0.8, 0.85, 0.9), steps=30000, n=100, W=4.0):
    """Liquid slab between z = 0.25 N_z and 0.75 N_z (tanh profiles of width
    W), a = 0.5, sigma = 0.116; densities at the slab centre and half a
    period away after `steps`."""
    import lbm_inputs as li
    out = []
    z = np.arange(n, dtype=np.float64)
    for t in temps:
        rl, rv = li.coexistence(t)
        prof = rv + 0.5 * (rl - rv) * (np.tanh(2.0 * (z - 0.25 * n) / W) - np.tanh(2.0 * (z - 0.75 * n) / W))
        rho = np.repeat(prof, n * n)
        cfg = _params(n, T_over_Tc=t, eos_a=0.5, sigma=0.116, tau_nu=0.8, storage="f64", **PAPER_RATES)
        lat = _lattice(cfg)
        lat.init_fields(rho, np.zeros((3, rho.size)))
        lat.step(steps)
        r = lat.read_fields()["rho"].cpu().numpy().reshape(n, n, n)
        d = lat.diagnostics()
        lat.close()
        col = r.mean(axis=(1, 2))
        out.append(_emit(dict(study="flat", T_over_Tc=t, steps=steps, rho_L=float(col[n // 2]), rho_V=float(col[0]),
                              maxwell_rho_L=rl, maxwell_rho_V=rv, max_u=d["max_u"], nonfinite=d["nonfinite"])))
    return out


def table2(ops=("nonorth", "orth"), nus=(0.01, 1.0 / 30.0, 0.05, 0.1, 0.15), steps=30000, n=120, storage="f64",
           warm_nu=0.1):
    """Cold start from the Eq. (59) profile at every viscosity.  A run whose
    cold start diverges is repeated from the state reached after `steps` at
    nu = warm_nu (same droplet, same lattice), then `steps` more at its own
    viscosity."""
    import lbm_inputs as li
    rl0, rv0 = li.coexistence(0.6)
    c = (n / 2, n / 2, n / 2)

    def cfg_for(op, nu):
        return _params(n, op=op, T_over_Tc=0.6, eos_a=0.25, sigma=0.105, tau_nu=tau_for_nu(nu), storage=storage,
                       **PAPER_RATES)

    out = []
    for op in ops:
        warm = None
        for nu in nus:
            t0 = time.time()
            lat = _lattice(cfg_for(op, nu))
            lat.init_droplets([dict(center=c, r0=40.0)], rl0, rv0, 5.0)
            lat.step(steps)
            obs = _droplet(lat, c, 40.0, 5.0)
            lat.close()
            out.append(_emit(dict(study="table2", op=op, nu=nu, inv_s_nu=tau_for_nu(nu), steps=steps, start="cold",
                                  seconds=round(time.time() - t0, 1), **obs)))
            if not obs["nonfinite"]:
                continue
            if warm is None:
                w = _lattice(cfg_for(op, warm_nu))
                w.init_droplets([dict(center=c, r0=40.0)], rl0, rv0, 5.0)
                w.step(steps)
                warm = w.save_state()
                w.close()
            lat = _lattice(cfg_for(op, nu))
            lat.load_state(warm)
            lat.step(steps)
            obs = _droplet(lat, c, 40.0, 5.0)
            lat.close()
            out.append(_emit(dict(study="table2", op=op, nu=nu, inv_s_nu=tau_for_nu(nu), steps=steps,
                                  start=f"state after {steps} steps at nu={warm_nu}", **obs)))
    return out


ORTH_READINGS = {
    # name: extra parameters of the orthogonal operator
    "meq_Morth_sigma_e_eps": dict(orth_meq=0, orth_sigma=1),
    "meq_Morth_sigma_e": dict(orth_meq=0, orth_sigma=0),
    "meq_tuned_sigma_e_eps": dict(orth_meq=1, orth_sigma=1),
    "meq_tuned_sigma_e": dict(orth_meq=1, orth_sigma=0),
    "meq_Morth_sigma_e_eps_seps_se": dict(orth_meq=0, orth_sigma=1, s_eps="s_e"),
    "meq_Morth_sigma_e_sm198": dict(orth_meq=0, orth_sigma=0, s_m=1.98),
    "meq_Morth_sigma_e_spi_snu": dict(orth_meq=0, orth_sigma=0, s_pi="s_nu", s_eps="s_nu"),
}


def orth_readings(readings=tuple(ORTH_READINGS), nus=(0.01, 0.05, 0.1, 0.15), steps=30000, n=120, warm_nu=0.1,
                  stab_nus=(1e-3, 2e-3), stab_steps=8000, chunk=250, seed=1805):
    """Readings of the orthogonal comparison operator against the two
    observations the paper prints for it: Table II (C-S at T = 0.6 T_c, the
    120^3 droplet, rho_V rising with nu: 0.00313 / 0.00319 / 0.00321 /
    0.00323) and the stability of the Table I phase separation at
    nu = 2e-3 (diverging at 1e-3).  Table II runs start cold except at
    nu = 0.01, which continues the nu = 0.1 state (a cold start diverges for
    every reading, as for the non-orthogonal model)."""
    import lbm_inputs as li
    rl0, rv0 = li.coexistence(0.6)
    c = (n / 2, n / 2, n / 2)
    out = []
    for name in readings:
        def rates(nu):
            extra = dict(ORTH_READINGS[name])
            for k, v in list(extra.items()):
                if v == "s_e":
                    extra[k] = PAPER_RATES["s_e"]
                elif v == "s_nu":
                    extra[k] = 1.0 / tau_for_nu(nu)
            return {**PAPER_RATES, **extra}

        def cfg_for(nu):
            return _params(n, op="orth", T_over_Tc=0.6, eos_a=0.25, sigma=0.105, tau_nu=tau_for_nu(nu),
                           storage="f64", **rates(nu))
        warm = None
        for nu in sorted(nus, reverse=True):
            lat = _lattice(cfg_for(nu))
            start = "cold"
            if nu < 0.05 and warm is not None:
                lat.load_state(warm)
                start = f"state after {steps} steps at nu={warm_nu}"
            else:
                lat.init_droplets([dict(center=c, r0=40.0)], rl0, rv0, 5.0)
            lat.step(steps)
            obs = _droplet(lat, c, 40.0, 5.0)
            if nu == warm_nu:
                warm = lat.save_state()
            lat.close()
            out.append(_emit(dict(study="orth_readings", reading=name, table="II", nu=nu, start=start, **obs)))
        for nu in stab_nus:
            cfg = _params(n, op="orth", tau_nu=tau_for_nu(nu), storage="f64", **EXP_PSI, **rates(nu))
            lat = _phase_separation_cfg(cfg, seed)
            diverged = None
            for k in range(stab_steps // chunk):
                lat.step(chunk)
                d = lat.diagnostics()
                if d["nonfinite"] or not math.isfinite(d["max_u"]) or d["max_u"] > 0.5:
                    diverged = (k + 1) * chunk
                    break
            lat.close()
            out.append(_emit(dict(study="orth_readings", reading=name, table="stability", nu=nu,
                                  steps=stab_steps, diverged_by_step=diverged, max_u=d["max_u"])))
    return out


def viscosity_ratio(ops=("nonorth", "orth"), ratios=(1.0, 2.0, 5.0, 10.0), nu_L=0.01, steps=30000, n=120,
                    warm_nu=0.1):
    """Sec. IV.D after Fig. 6: the Table II droplet with liquid viscosity
    nu_L = 0.01 and vapour viscosity nu_ratio nu_L, nu linear in rho between
    the coexistence densities (the library's reading); maximum spurious
    velocity against nu_V / nu_L.  A run whose cold start diverges restarts
    from the state reached after `steps` at uniform nu = warm_nu."""
    import lbm_inputs as li
    rl0, rv0 = li.coexistence(0.6)
    c = (n / 2, n / 2, n / 2)

    def cfg_for(op, ratio, nu):
        return _params(n, op=op, T_over_Tc=0.6, eos_a=0.25, sigma=0.105, tau_nu=tau_for_nu(nu), storage="f64",
                       nu_ratio=ratio, visc_rho_L=rl0, visc_rho_V=rv0, **PAPER_RATES)

    out = []
    for op in ops:
        warm = None
        for ratio in ratios:
            lat = _lattice(cfg_for(op, ratio, nu_L))
            lat.init_droplets([dict(center=c, r0=40.0)], rl0, rv0, 5.0)
            lat.step(steps)
            obs = _droplet(lat, c, 40.0, 5.0)
            lat.close()
            start = "cold"
            if obs["nonfinite"]:
                if warm is None:
                    w = _lattice(cfg_for(op, 1.0, warm_nu))
                    w.init_droplets([dict(center=c, r0=40.0)], rl0, rv0, 5.0)
                    w.step(steps)
                    warm = w.save_state()
                    w.close()
                lat = _lattice(cfg_for(op, ratio, nu_L))
                lat.load_state(warm)
                lat.step(steps)
                obs = _droplet(lat, c, 40.0, 5.0)
                lat.close()
                start = f"state after {steps} steps at nu={warm_nu}"
            out.append(_emit(dict(study="viscosity_ratio", op=op, nu_L=nu_L, nu_ratio=ratio, steps=steps,
                                  start=start, **obs)))
    return out


def _cavity_cfg(L, U, Re, op, storage):
    """Lid-driven cavity of Appendix B: L^3, walls on all faces, the face
    y = L - 1/2 moving along x at U, nu = U L / Re, single phase (G = 0),
    s_e = 0.8 and the other non-conserved rates 1.2 as in Sec. IV."""
    nu = U * L / Re
    return _params(L, op=op, storage=storage, psi_form="exp", G=0.0, sigma=0.0, tau_nu=tau_for_nu(nu),
                   wall_x=1, wall_y=1, wall_z=1, lid_u=(U, 0.0, 0.0), lid_rho=1.0, **PAPER_RATES)


def cavity_cost(sizes=(60, 80, 110), steps=5000, storages=("f64", "f32")):
    """Table III on the GPU: time of `steps` iterations of the cavity for
    both operators (HIP events around the step launches)."""
    import torch
    out = []
    for st in storages:
        for L in sizes:
            row = dict(study="cavity_cost", L=L, steps=steps, storage=st)
            for op in ("orth", "nonorth"):
                lat = _lattice(_cavity_cfg(L, 0.1, 400.0, op, st))
                lat.init_fields(np.ones(L ** 3), np.zeros((3, L ** 3)))
                lat.step(20)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                lat.step(steps)
                e1.record()
                torch.cuda.synchronize()
                sec = e0.elapsed_time(e1) / 1e3
                row[f"t_{op}_s"] = round(sec, 4)
                row[f"mlups_{op}"] = round(L ** 3 * steps / sec / 1e6, 1)
                lat.close()
            row["t_orth_over_t_nonorth_minus_1"] = round(row["t_orth_s"] / row["t_nonorth_s"] - 1, 4)
            out.append(_emit(row))
    return out


def throughput():
    """GPU MLUPS for each standard workload: 32^3 droplet (FP64), 128^3
    Laplace droplet (FP64, FP32), 256^3 two droplets (FP64, FP32, F16S,
    F16N), 384 x 384 x 192 sessile droplet (FP32, F16N), and the 256-run batch (FP32, F16S,
    F16N), with the kernels and tiles of ``tuning``.  (The oracle's rates on
    the host for the same workloads come from ``bench.py --cpu-workloads``.)"""
    import torch

    import lbm_inputs as li
    from paper_1805_08643_amd import tuning
    from paper_1805_08643_amd.binding import Batch, f16_exp_for
    work = [("droplet_32", li.c1_droplet, ("f64",), 500),
            ("laplace_128", lambda: li.c2_laplace(24), ("f64", "f32"), 200),
            ("two_droplets_256", li.c3_two_droplets, ("f64", "f32", "f16s", "f16n"), 200),
            ("sessile_384x384x192", lambda: li.c4_sessile(60.0), ("f32", "f16n"), 200)]
    out = []
    for name, fn, storages, gsteps in work:
        cfg, init = fn()
        row = dict(study="throughput", workload=name, nodes=cfg["nx"] * cfg["ny"] * cfg["nz"])
        for st in storages:
            c = dict(cfg, storage=st, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
            lat = _lattice(c)
            mode = tuning.mode_for(name, st)
            lat.set_step_mode(mode)
            tile = tuning.tile_for(name, st, mode)
            if tile:
                lat.set_tile(*tile)
            lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
            lat.step(10)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lat.step(gsteps)
            e1.record()
            torch.cuda.synchronize()
            row[f"gpu_{st}_mlups"] = round(row["nodes"] * gsteps / (e0.elapsed_time(e1) * 1e-3) / 1e6, 1)
            lat.close()
        out.append(_emit(row))
    runs = li.c5_batch()
    row = dict(study="throughput", workload="batch_256_runs")
    for st in ("f32", "f16s", "f16n"):
        cfgs = [dict(pp, storage=st, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
                for pp, init in runs]
        b = Batch(cfgs)
        for k, (_, init) in enumerate(runs):
            b.init_droplets(k, init["droplets"], init["rho_L"], init["rho_V"], init["W"])
        b.autotune(2)
        b.step(20, 10)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(50, 10)
        e1.record()
        torch.cuda.synchronize()
        row["nodes"] = b.nodes
        row[f"gpu_{st}_mlups"] = round(b.nodes * 50 / (e0.elapsed_time(e1) * 1e-3) / 1e6, 1)
        b.close()
        del b
        torch.cuda.empty_cache()
    out.append(_emit(row))
    return out


def laplace_cs(ops=("nonorth", "orth"), storages=("f64", "f32"), radii=(24, 28, 32, 36, 40), steps=20000):
    """Radii from 24: droplets of radius 12 to 20 evaporate in the 128^3 box
    (Kelvin effect, as in `laplace`)."""
    import lbm_inputs as li
    out = {}
    for st in storages:
        for op in ops:
            pts = []
            for r0 in radii:
                cfg, init = li.c2_laplace(r0, op=op)
                c = init["droplets"][0]["center"]
                lat = _lattice(dict(cfg, storage=st))
                lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
                lat.step(steps)
                pts.append(_emit(dict(study="laplace_cs", op=op, storage=st, r0=r0,
                                      **_droplet(lat, c, float(r0), init["W"]))))
                lat.close()
            x = np.array([1.0 / p["R_d"] for p in pts])
            y = np.array([p["dp"] for p in pts])
            slope, icpt, r2 = _linfit(x, y)
            out[f"{op}_{st}"] = _emit(dict(study="laplace_cs_fit", op=op, storage=st, slope=slope,
                                           surface_tension=slope / 2, intercept=icpt, r2=r2,
                                           max_dp=float(y.max()), steps=steps, points=pts))
    return out


def precision_results(storages=("f64", "f32", "f16s", "f16n"), radii=(24, 32, 40), steps=20000):
    """Error of each storage format against FP64 storage per result, on the
    128^3 Laplace droplets (C-S EOS at T = 0.7 T_c, density ratio 38.5) run to
    rest: the coexistence densities rho_L and rho_V, the pressure jump Delta p
    of each radius and the surface tension from the Laplace fit, the
    spurious-current magnitude max |u|, and the density field (largest
    relative difference over the lattice).  F16S shifts by rho_V; F16N by the
    binary16 density of the node that pulls each population."""
    import torch

    import lbm_inputs as li
    from paper_1805_08643_amd.binding import f16_exp_for
    out, runs, fields = [], {}, {}
    for st in storages:
        for r0 in radii:
            cfg, init = li.c2_laplace(r0)
            c = init["droplets"][0]["center"]
            lat = _lattice(dict(cfg, storage=st, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"])))
            lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
            lat.step(steps)
            runs[(st, r0)] = _droplet(lat, c, float(r0), init["W"])
            fields[(st, r0)] = lat.read_fields()["rho"].cpu()
            lat.close()
        x = np.array([1.0 / runs[(st, r)]["R_d"] for r in radii])
        y = np.array([runs[(st, r)]["dp"] for r in radii])
        runs[(st, "fit")] = dict(zip(("slope", "intercept", "r2"), _linfit(x, y)))
    rel = lambda a, b: abs(a - b) / abs(b)
    for st in storages:
        row = dict(study="precision_results", storage=st, steps=steps, radii=list(radii),
                   surface_tension=runs[(st, "fit")]["slope"] / 2, laplace_r2=runs[(st, "fit")]["r2"], per_radius=[])
        for r0 in radii:
            a, b = runs[(st, r0)], runs[("f64", r0)]
            d = dict(r0=r0, **{k: a[k] for k in ("rho_L", "rho_V", "dp", "R_d", "max_u")})
            if st != "f64":
                f, g = fields[(st, r0)], fields[("f64", r0)]
                d.update(rho_L_rel_err=rel(a["rho_L"], b["rho_L"]), rho_V_rel_err=rel(a["rho_V"], b["rho_V"]),
                         dp_rel_err=rel(a["dp"], b["dp"]), max_u_rel_err=rel(a["max_u"], b["max_u"]),
                         rho_field_max_rel_err=float(((f - g).abs() / g).max()))
            row["per_radius"].append(d)
        if st != "f64":
            row["surface_tension_rel_err"] = rel(row["surface_tension"], runs[("f64", "fit")]["slope"] / 2)
        out.append(_emit(row))
    torch.cuda.empty_cache()
    return out


def precision(steps=(100, 500, 1000, 2000), n=256, crop=64):
    """Density error of FP32 and 16-bit storage against FP64 storage on the
    central crop^3 box, the droplet-pair observables, and the relative mass
    drift of each run.  Shifted FP16 runs with the default shift
    rho_ref = rho_V ("f16s") and the two control shifts, rho_ref = 0
    ("f16s_rho0", unshifted) and rho_ref = (rho_L + rho_V) / 2 ("f16s_mid");
    "f16n" shifts every population by the binary16 density of the node that
    pulls it."""
    import torch

    import lbm_inputs as li
    from paper_1805_08643_amd.binding import f16_exp_for
    if isinstance(steps, int):
        steps = (steps,)
    cfg, init = li.c3_two_droplets(n=n)
    shifts = {"f16s": init["rho_V"], "f16s_rho0": 0.0, "f16s_mid": 0.5 * (init["rho_L"] + init["rho_V"])}
    variants = ("f32", "f16s", "f16s_rho0", "f16s_mid", "f16n")
    lats = {}
    for st in ("f64",) + variants:
        c = dict(cfg, storage="f16s" if st.startswith("f16s") else st, rho_ref=shifts.get(st, init["rho_V"]),
                 f16_exp=f16_exp_for(1.25 * init["rho_L"]))
        lat = _lattice(c)
        lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
        lats[st] = lat
    m0 = {st: lat.diagnostics()["mass"] for st, lat in lats.items()}
    lo = n // 2 - crop // 2
    center = (n / 2, n / 2, n / 2)
    out = []
    done = 0
    for s in steps:
        fields, obs = {}, {}
        for st, lat in lats.items():
            lat.step(s - done)
            rho = lat.read_fields()["rho"].reshape(n, n, n)[lo:lo + crop, lo:lo + crop, lo:lo + crop].double()
            fields[st] = rho.cpu()
            d = lat.diagnostics(center=center, r_in=10.0, r_out=80.0)
            obs[st] = dict(rho_center=d["rho_in"] / max(d["n_in"], 1), rho_far=d["rho_out"] / max(d["n_out"], 1),
                           dp=d["p_in"] / max(d["n_in"], 1) - d["p_out"] / max(d["n_out"], 1), max_u=d["max_u"],
                           mass_drift=(d["mass"] - m0[st]) / m0[st])
        done = s
        ref = fields["f64"]
        liquid = ref > 0.5 * (init["rho_L"] + init["rho_V"])
        row = dict(study="precision", step=s, f64=obs["f64"], rho_ref=shifts)
        for st in variants:
            rel = (fields[st] - ref).abs() / ref
            row[st] = dict(rho_max_rel_err_liquid=float(rel[liquid].max()) if bool(liquid.any()) else None,
                           rho_max_rel_err_vapour=float(rel[~liquid].max()),
                           rho_mean_rel_err=float(rel.mean()), mass_drift=obs[st]["mass_drift"],
                           **{f"{k}_rel_err": abs(obs[st][k] - obs["f64"][k]) / abs(obs["f64"][k])
                              for k in ("rho_center", "rho_far", "dp", "max_u")})
        out.append(_emit(row))
    for lat in lats.values():
        lat.close()
    torch.cuda.empty_cache()
    return out


STUDIES = {f.__name__: f for f in (table1, stability, laplace, spurious, contact, flat, table2, orth_readings,
                                   viscosity_ratio,
                                   cavity_cost, laplace_cs, contact_cs, contact_precision, precision,
                                   precision_results, storage_drift,
                                   throughput)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("studies", nargs="+", choices=sorted(STUDIES))
    ap.add_argument("--out-dir")
    ap.add_argument("--steps", type=int)
    a = ap.parse_args(argv)
    res = {}
    for name in a.studies:
        kw = {"steps": a.steps} if a.steps else {}
        t0 = time.time()
        try:
            res[name] = STUDIES[name](**kw)
        except (ValueError, np.linalg.LinAlgError, ZeroDivisionError) as e:
            res[name] = {"error": f"{type(e).__name__}: {e}"}
        print(f"[study] {name} done in {time.time() - t0:.1f} s", flush=True)
        if a.out_dir:
            os.makedirs(a.out_dir, exist_ok=True)
            with open(os.path.join(a.out_dir, f"{name}.json"), "w") as fh:
                json.dump(res[name], fh, indent=1)
    return res


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
