"""Multi-step parity at full size, in the launch configuration the benchmark
times: every population of the whole lattice against the FP64 oracle.

* 256^3 two-droplet workload (the benchmark workload: Sec. IV.D setup, two
  Eq. (59) droplets approaching), FP32 storage and arithmetic in the split
  step with its tuned tile and streaming stores, 50 steps: the density field
  and every population within the stated FP32 bound of 1e-5 relative to the
  node's density.
* 384 x 384 x 192 sessile droplet between wetting walls (Eq. (57), gravity),
  FP64, 30 steps: every population within 1e-12.

* 256^3 two-droplet workload, 100 steps (to the droplets' contact), FP32,
  F16S and F16N storage in their benchmark launch shapes against the FP64
  oracle itself: the density field within 1e-5 (FP32) and within the 16-bit
  caps of 2e-3 in the liquid and 5e-3 in the vapour (F16N); F16S's errors are
  reported (they exceed the caps on this workload, as the precision study
  shows against FP64 storage).

The oracle runs on up to 16 host threads; each case takes it 40-80 s.
"""
import os

import numpy as np
import pytest
import torch

import lbm_inputs as li
from oracle import ref
from paper_1805_08643_amd import tuning
from paper_1805_08643_amd.binding import Lattice

pytestmark = pytest.mark.gpu


def _threads():
    return min(16, os.cpu_count() or 1)


def _gpu_run(cfg, rho, u, steps, mode, tile):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"[gpu] full size {cfg['nx']}x{cfg['ny']}x{cfg['nz']} {cfg['storage']} mode={mode} tile={tile} "
          f"steps={steps}", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode(mode)
    if tile:
        lat.set_tile(*tile)
    lat.init_fields(rho, u).step(steps)
    d = lat.diagnostics()
    got = lat.read_populations().cpu().numpy()
    lat.close()
    torch.cuda.empty_cache()
    assert d["status"] == 0 and d["nonfinite"] == 0
    return got


def _rel_err(got, want):
    r = want.sum(0)
    pop = 0.0
    for a in range(19):  # one direction at a time keeps the temporaries small
        pop = max(pop, float((np.abs(got[a] - want[a]) / r).max()))
    rho = float((np.abs(got.sum(0) - r) / r).max())
    return pop, rho


def test_fp32_split_50_steps_two_droplets_256():
    cfg, init = li.c3_two_droplets()
    cfg = dict(cfg, storage="f32")
    rho, u = li.init_fields(cfg, init)
    mode = tuning.mode_for("two_droplets_256", "f32")
    tile = tuning.tile_for("two_droplets_256", "f32", mode)
    assert mode == "split"
    got = _gpu_run(cfg, rho, u, 50, mode, tile)
    p = ref.make_params(cfg, nthreads=_threads())
    want = ref.step(p, ref.equilibrium(p, rho, u), 50)
    pop, dens = _rel_err(got, want)
    print(f"  50 steps: population err {pop:.3e}, density err {dens:.3e} (bound 1e-5)", flush=True)
    assert pop < 1e-5 and dens < 1e-5


def test_fp64_30_step_prefix_sessile_384x384x192():
    cfg, init = li.c4_sessile(60.0)
    cfg = dict(cfg, storage="f64")
    rho, u = li.init_fields(cfg, init)
    mode = tuning.mode_for("sessile_384x384x192", "f64")
    tile = tuning.tile_for("sessile_384x384x192", "f64", mode)
    got = _gpu_run(cfg, rho, u, 30, mode, tile)
    p = ref.make_params(cfg, nthreads=_threads())
    want = ref.step(p, ref.equilibrium(p, rho, u), 30)
    pop, dens = _rel_err(got, want)
    print(f"  30 steps: population err {pop:.3e}, density err {dens:.3e} (bound 1e-12)", flush=True)
    assert pop < 1e-12


def test_storage_formats_100_steps_against_oracle_two_droplets_256():
    cfg, init = li.c3_two_droplets()
    rho, u = li.init_fields(cfg, init)
    p = ref.make_params(dict(cfg, storage="f64"), nthreads=_threads())
    print("[oracle] 256^3 two droplets, 100 steps", flush=True)
    want = ref.step(p, ref.equilibrium(p, rho, u), 100).sum(0)
    del p
    liquid = want > 0.5 * (init["rho_L"] + init["rho_V"])
    from paper_1805_08643_amd.binding import f16_exp_for
    errs = {}
    for st in ("f32", "f16s", "f16n"):
        c = dict(cfg, storage=st, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
        mode = tuning.mode_for("two_droplets_256", st)
        tile = tuning.tile_for("two_droplets_256", st, mode)
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        print(f"[gpu] 256^3 two droplets {st} mode={mode} tile={tile} 100 steps", flush=True)
        lat = Lattice(c)
        lat.set_step_mode(mode)
        if tile:
            lat.set_tile(*tile)
        lat.init_fields(rho, u).step(100)
        got = lat.read_fields()["rho"].cpu().numpy()
        lat.close()
        torch.cuda.empty_cache()
        rel = np.abs(got - want) / want
        errs[st] = (float(rel[liquid].max()), float(rel[~liquid].max()))
        print(f"  {st}: density err liquid {errs[st][0]:.2e}, vapour {errs[st][1]:.2e}", flush=True)
    assert max(errs["f32"]) < 1e-5
    assert errs["f16n"][0] < 2e-3 and errs["f16n"][1] < 5e-3

