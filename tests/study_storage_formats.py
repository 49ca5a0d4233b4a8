"""CPU study of 16-bit population storage on a scaled two-droplet collision.

The oracle's FP64 step (Eqs. 5-16) runs unchanged; after every step the
state it hands on is rounded as a storage format would round it, so the run
sees exactly the storage error and nothing else.  Formats:

* ``f32``: every population rounded to binary32.
* ``f16s``, ``f16s_rho0``, ``f16s_mid``: the library's F16S format,
  h = (f_a - w_a rho_ref) 2^E in binary16 with one reference density for the
  whole lattice (the vapour density, zero, or the mean of the two
  coexistence densities).
* ``f16n``: binary16 of h = (f_a(x) - w_a rho~(x)) 2^E, where rho~(x) is the
  density the node x had one step earlier, itself rounded to binary16.  The
  reference follows every node, so h holds only what changed at the node
  during one step (the streaming of a moving or curved interface, the
  velocity moments and the non-equilibrium part) instead of the whole
  liquid-vapour contrast.  This is the first form of F16N: the shift in
  FP32, the loaded value rounded to FP32, stores rounded to nearest.
* ``f16n_sr``: the library's F16N: exact loads (w_a rt + h 2^-E), each store
  rounded stochastically with the step's dither (``round_trip_n_sr`` of
  ``f16s_format``).  Rounding to nearest let values that change by less
  than half a binary16 unit per step stagnate; the dither removes that bias.

Run from the repository root (about 25 minutes on 8 threads at n = 64):

    python tests/study_storage_formats.py --n 64 --steps 50,100,200,400

``--formats f16n_sr --merge`` adds formats to an existing results file.

Writes ``results/storage_formats_emulated.json``: for every format and step
the largest relative density error in the liquid and in the vapour of the
central box (side n/4), and the relative mass drift, against the FP64 run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import lbm_inputs as li  # noqa: E402
from oracle import ref  # noqa: E402
from tests import f16s_format as fmt  # noqa: E402

# Lattice weights of D3Q19 (rest, six axis, twelve diagonal directions), in
# the oracle's direction order.
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None]


def to_f32(x):
    return x.astype(np.float32).astype(np.float64)


def to_f16(x):
    return x.astype(np.float16).astype(np.float64)


def shifted(f, ref_rho, E):
    """Binary16 of (f - w rho_ref) 2^E, decoded back; rho_ref is a scalar or a
    per-node array."""
    shift = to_f32(W * ref_rho)
    return to_f32(to_f16((to_f32(f) - shift) * 2.0 ** E) / 2.0 ** E + shift)


def store(name, f, rho_prev, rho_l, rho_v, E, cfg=None, seed=None):
    """The state f after the storage of format `name`; seed: the step's
    rounding seed (None: the initial write)."""
    if name == "f16n_sr":
        c = dict(cfg, f16_exp=E)
        return fmt.round_trip_n(f, rho_prev, c) if seed is None else fmt.round_trip_n_sr(f, rho_prev, c, seed)
    if name == "f64":
        return f
    if name == "f32":
        return to_f32(f)
    if name == "f16s":
        return shifted(f, rho_v, E)
    if name == "f16s_rho0":
        return shifted(f, 0.0, E)
    if name == "f16s_mid":
        return shifted(f, 0.5 * (rho_l + rho_v), E)
    if name == "f16n":
        return shifted(f, to_f16(rho_prev)[None, :], E)
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", default="50,100,200,400")
    ap.add_argument("--formats", default="f32,f16s,f16s_rho0,f16s_mid,f16n")
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(ROOT, "results", "storage_formats_emulated.json"))
    ap.add_argument("--merge", action="store_true", help="keep the other formats of an existing --out file")
    a = ap.parse_args()
    n = a.n
    steps = [int(s) for s in a.steps.split(",")]
    cfg, init = li.c3_two_droplets(n=n)
    rho, u = li.init_fields(cfg, init)
    p = ref.make_params(cfg, nthreads=a.threads)
    rl, rv = init["rho_L"], init["rho_V"]
    # 2^E keeps the largest |h| (a rest population of 1.25 rho_L against
    # rho_ref = 0) below 2^15, the scale the library picks for F16S.
    E = int(np.floor(np.log2(2.0 ** 15 / (1.25 * rl / 3.0))))
    f0 = ref.equilibrium(p, rho, u)
    c, h = n // 2, n // 8
    box = (slice(c - h, c + h),) * 3
    runs, out = {}, {"study": "storage_formats_emulated", "workload": f"two droplets, {n}^3 (the 256^3 recipe scaled)",
                     "scale_exponent": E, "steps": steps, "formats": {}}
    for name in ["f64"] + a.formats.split(","):
        t0 = time.time()
        f = store(name, f0, f0.sum(0), rl, rv, E, cfg)
        done, rec = 0, {}
        for s in steps:
            for t in range(done, s):
                rp = f.sum(0)
                f = store(name, ref.step(p, f, 1), rp, rl, rv, E, cfg, seed=t)
            done = s
            rec[s] = f.sum(0).copy()
        runs[name] = rec
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)
        if name == "f64":
            continue
        rows = []
        for s in steps:
            w, g = runs["f64"][s], rec[s]
            w3, g3 = w.reshape(n, n, n)[box].ravel(), g.reshape(n, n, n)[box].ravel()
            rel = np.abs(g3 - w3) / w3
            liq = w3 > 0.5 * (rl + rv)
            rows.append(dict(step=s, rho_max_rel_err_liquid=float(rel[liq].max()) if liq.any() else 0.0,
                             rho_max_rel_err_vapour=float(rel[~liq].max()),
                             mass_drift=float((g.sum() - w.sum()) / w.sum())))
            print(f"  step {s}: liquid {rows[-1]['rho_max_rel_err_liquid']:.2e} vapour "
                  f"{rows[-1]['rho_max_rel_err_vapour']:.2e} mass {rows[-1]['mass_drift']:+.1e}", flush=True)
        out["formats"][name] = rows
    if a.merge and os.path.exists(a.out):
        with open(a.out) as fh:
            old = json.load(fh)
        if old.get("steps") == steps and old.get("scale_exponent") == E:
            old["formats"].update(out["formats"])
            out = old
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
