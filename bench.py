"""Benchmark of the fused D3Q19 MRT pseudopotential step on one MI355X.

Default workload: the 256^3 periodic two-droplet precision study (C-S EOS at
T = 0.6 T_c, a = 0.25, droplets of radius 30 approaching at 0.05), FP32
population storage, non-orthogonal operator.  One step = one lattice update
of every node (all of the fused kernel's work).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32|f16s|f16n|f64]
                  [--op nonorth|orth] [--no-cpu] [--no-variants]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % of HBM roofline; FP32/FP16-storage vs FP64 at stated error"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
WORKLOAD = "two_droplets_256"
WORKLOADS = {
    "two_droplets_256": "256^3 periodic, two droplets r0=30 approaching at 0.05, C-S T=0.6Tc a=0.25, sigma=0.105",
    "sessile_384x384x192": "384x384x192, periodic x and y, half-way bounce-back walls in z with the Eq. (57) "
                           "wetting layer at 60 deg, sessile droplet r0=40, C-S T=0.7Tc, gravity 1e-6",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16s", "f16n", "f64"])
    ap.add_argument("--op", default="nonorth", choices=["nonorth", "orth"])
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(WORKLOADS) + ["batch_256"],
                    help="lattice to time (default: the 256^3 two-droplet workload); batch_256 times only the "
                         "256-run batch")
    ap.add_argument("--mode", default=None, choices=["fused", "pairs", "quads", "split"],
                    help="step kernel; default: the faster one measured for the storage")
    ap.add_argument("--tile", default=None, help="launch shape tx,ty,cz instead of the tuned one")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-workloads", action="store_true",
                    help="only time the oracle on the host for every standard workload (one JSON line each)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the hand-written 1 GiB device copy 5 times (HBM counter calibration)")
    ap.add_argument("--ceiling-probe", action="store_true",
                    help="only run the data-movement probes (flat copy, 19-plane streaming, tile march) at the "
                         "byte volume of the FP32 256^3 step and print their rates")
    return ap.parse_args()


def _timed(launch, reps):
    """Mean ms of `launch` over reps launches, HIP events on torch's current
    stream (the stream the probes are launched on)."""
    import torch
    launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_probe(reps=5, quiet=False, nbytes=1 << 30, streaming=True, blocks=32768):
    """A hand-written device copy of known size (16-byte accesses, 32768
    blocks of 256 threads, streaming stores): 1 GiB read + 1 GiB written per
    launch, used to scale the HBM byte counters of rocprofv3 and as the
    practical read+write rate of the part."""
    import torch

    from paper_1805_08643_amd import probe
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream().cuda_stream
    ms = _timed(lambda: probe.lbm_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, streaming, blocks, st), reps)
    out = {"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "streaming_stores": streaming,
           "ms_per_copy": round(ms, 4), "GBps_read_plus_write": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}
    assert torch.equal(src[:1024], dst[:1024])
    del src, dst
    torch.cuda.empty_cache()
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


def ceiling_probe(reps=10, quick=False, storage="f32"):
    """Rates of pure data movement at the byte volume of one step of the
    256^3 lattice (19 planes of 256^3 values: 1.27 GB read and 1.27 GB
    written in FP32, half that in F16S), in the access patterns of the step
    kernels.  quick: only the fastest flat copy and 19-plane stream
    (streaming stores)."""
    import torch

    from paper_1805_08643_amd import probe
    n, s = 256, (2 if storage == "f16s" else 4)
    plane_bytes = n ** 3 * s
    total = 19 * plane_bytes
    src = torch.ones(total // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream().cuda_stream
    rows = []

    def rec(kind, ms, **kw):
        rows.append({"probe": kind, **kw, "ms": round(ms, 4),
                     "GBps_read_plus_write": round(2 * total / (ms * 1e-3) / 1e9, 1),
                     "frac_of_8TBps": round(2 * total / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)})

    if quick:
        ms = _timed(lambda: probe.lbm_probe_copy(src.data_ptr(), dst.data_ptr(), total, 1, 32768, st), reps)
        rec("flat_copy_16B", ms, streaming_stores=1, blocks=32768)
        ms = _timed(lambda: probe.lbm_probe_stream19(src.data_ptr(), dst.data_ptr(), plane_bytes, 8, 1, 0, st), reps)
        rec("stream19", ms, group_bytes=8, streaming_stores=1, blocks=8192)
    for nt in (() if quick else (0, 1)):
        for blocks in (2048, 8192, 32768):
            ms = _timed(lambda: probe.lbm_probe_copy(src.data_ptr(), dst.data_ptr(), total, nt, blocks, st), reps)
            rec("flat_copy_16B", ms, streaming_stores=nt, blocks=blocks)
        for gb in (8, 16):
            ms = _timed(lambda: probe.lbm_probe_stream19(src.data_ptr(), dst.data_ptr(), plane_bytes, gb, nt, 0, st),
                        reps)
            rec("stream19", ms, group_bytes=gb, streaming_stores=nt, blocks=8192)
        # the split step's tiles: FP32 128 x 4 nodes (64 x 4 groups of two) with z runs of 128 planes,
        # F16S 128 x 8 nodes (32 x 8 groups of four) with z runs of 64
        tiles = ((8, 64, 4, 128), (16, 32, 4, 128), (8, 64, 8, 64), (8, 128, 2, 128)) if s == 4 else \
            ((8, 32, 8, 64), (16, 16, 8, 64), (8, 64, 4, 64), (8, 64, 4, 128))
        for gb, tx, ty, cz in tiles:
            nodes_per_group = gb // s
            ms = _timed(lambda: probe.lbm_probe_march19(src.data_ptr(), dst.data_ptr(), n // nodes_per_group, n, n,
                                                        gb, tx, ty, cz, nt, st), reps)
            rec("march19", ms, group_bytes=gb, tile_groups=[tx, ty, cz], tile_nodes=[tx * nodes_per_group, ty, cz],
                streaming_stores=nt)
    assert torch.equal(src[-1024:], dst[-1024:])
    del src, dst
    torch.cuda.empty_cache()
    return {"storage": storage, "bytes_read": total, "bytes_written": total, "rows": rows,
            "best_GBps": max(r["GBps_read_plus_write"] for r in rows)}


def make_lattice(storage, op, mode=None, workload=WORKLOAD, tile=None):
    import lbm_inputs as li
    from paper_1805_08643_amd import tuning
    from paper_1805_08643_amd.binding import Lattice, f16_exp_for
    if workload == "sessile_384x384x192":
        cfg, init = li.c4_sessile(60.0)
        cfg = dict(cfg, op=op)
    else:
        cfg, init = li.c3_two_droplets(op=op)
    cfg = dict(cfg, storage=storage, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
    lat = Lattice(cfg, "cuda:0")
    mode = mode or tuning.mode_for(workload, storage)
    lat.set_step_mode(mode)
    tile = tile or tuning.tile_for(workload, storage, mode)
    if tile:
        lat.set_tile(*tile)
    lat.mode = mode
    lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
    return lat, cfg, init


def time_steps(lat, steps, warmup, kernel_timing):
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    if kernel_timing:
        lat.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    kms = None
    if kernel_timing:
        kms, n = lat.kernel_time()
        assert n == steps, (n, steps)
        lat.set_timing(False)
    return ms, wall, kms


def precision_check(steps=100):
    """Errors of FP32, F16S and F16N storage against FP64 storage on the
    benchmark workload after `steps` steps from the same initial droplets:
    largest relative density error in the liquid and in the vapour over the
    whole lattice, and the relative mass drift; with the bounds the tests
    hold them to (density: 1e-5 for FP32, 2e-3 liquid / 5e-3 vapour for the
    16-bit formats)."""
    import torch
    out, ref = {"steps": steps, "reference": "FP64 storage on the GPU (matches the FP64 oracle to 1e-12)",
                "bounds": {"f32": 1e-5, "f16": {"liquid": 2e-3, "vapour": 5e-3}}}, None
    for st in ("f64", "f32", "f16s", "f16n"):
        lat, cfg, init = make_lattice(st, "nonorth")
        m0 = lat.diagnostics()["mass"]
        lat.step(steps)
        rho = lat.read_fields()["rho"]
        m1 = lat.diagnostics()["mass"]
        lat.close()
        del lat
        if ref is None:
            ref = rho
            liquid = ref > 0.5 * (init["rho_L"] + init["rho_V"])
        else:
            rel = (rho - ref).abs() / ref
            out[st] = {"rho_max_rel_err_liquid": float(rel[liquid].max()),
                       "rho_max_rel_err_vapour": float(rel[~liquid].max()),
                       "mass_drift": (m1 - m0) / m0}
            del rho, rel
        torch.cuda.empty_cache()
    return out


def bench_batch(storage, steps=40, graph_steps=10):
    """Batched workload: 256 independent periodic droplet runs, L ~ U{32, 48,
    64, 96}, T/Tc ~ U[0.6, 0.9], tau_nu ~ U[0.6, 1.2] (seed 1805), one
    persistent launch per step.  Aggregate MLUPS with plain launches, with
    hipGraph replay, and after the batch autotuner."""
    import torch

    import lbm_inputs as li
    from paper_1805_08643_amd.binding import Batch, algorithmic_bytes_per_node, f16_exp_for
    runs = li.c5_batch()
    cfgs = [dict(p, storage=storage, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
            for p, init in runs]
    b = Batch(cfgs)
    for k, (_, init) in enumerate(runs):
        b.init_droplets(k, init["droplets"], init["rho_L"], init["rho_V"], init["W"])
    N = b.nodes

    def timed(graph):
        b.step(2 * graph_steps, graph)  # warm-up (and graph capture)
        torch.cuda.synchronize()
        b.kernel_time()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(steps, graph)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        kms, _ = b.kernel_time()
        return ms, kms

    out = {"runs": len(runs), "nodes": N, "storage": storage, "step_mode": b.step_mode()}
    ms, _ = timed(0)
    out["mlups_plain_launches"] = round(N / (ms * 1e-3) / 1e6, 1)
    ms, _ = timed(graph_steps)
    out["mlups_graph"] = round(N / (ms * 1e-3) / 1e6, 1)
    blocks = b.autotune(3)
    ms, kms = timed(graph_steps)
    out["mlups_tuned_graph"] = round(N / (ms * 1e-3) / 1e6, 1)
    out["tuned_blocks"] = blocks
    out["tuned_step_mode"] = b.step_mode()
    out["ms_per_step"] = round(ms, 4)
    out["hbm_frac"] = round(algorithmic_bytes_per_node(storage) * N / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    d = b.read_fields(0)["rho"]
    out["finite"] = bool(torch.isfinite(d).all().item())
    b.close()
    del b
    torch.cuda.empty_cache()
    out["mlups_one_launch_per_run"] = round(per_run_launches(cfgs, runs, steps // 4), 1)
    return out


def per_run_launches(cfgs, runs, steps):
    """The same runs as separate lattices, one launch per run per step."""
    import torch

    from paper_1805_08643_amd.binding import Lattice
    lats = []
    for c, (_, init) in zip(cfgs, runs):
        lat = Lattice(c)
        lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
        lats.append(lat)
    N = sum(lat.N for lat in lats)
    for lat in lats:
        lat.step(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        for lat in lats:
            lat.step(1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for lat in lats:
        lat.close()
    del lats
    torch.cuda.empty_cache()
    return N / (ms * 1e-3) / 1e6


KERNEL_NAMES = {"fused": "k_step (fused psi/force + collide + pull-stream)",
                "pairs": "k_step2 (fused psi/force + collide + pull-stream, two nodes per thread)",
                "quads": "k_step4 (fused psi/force + collide + pull-stream, four nodes per thread)",
                "split": "k_step_split (psi/force + collide + pull-stream, 8-byte node groups, pulling and "
                         "colliding waves)"}


def read_traffic(storage, op, mode, workload=WORKLOAD):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it covers this kernel built from the current sources; None otherwise."""
    from paper_1805_08643_amd.build import source_digest
    kern = {"pairs": "step2", "quads": "step4", "split": "step_split"}.get(mode, "step")
    path = os.path.join(ROOT, "profiles", f"{kern}_{workload}_{storage}_{op}_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    d = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", txt)
    if not d or d.group(1) != source_digest():
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def cpu_baseline(cfg, init, budget_s):
    import numpy as np

    import lbm_inputs as li
    from oracle import ref
    threads = min(16, os.cpu_count() or 1)
    p = ref.make_params(cfg, nthreads=threads)
    rho, u = li.init_fields(cfg, init)
    f = ref.equilibrium(p, rho, u)
    N = rho.size
    t0 = time.perf_counter()
    f = ref.step(p, f, 1)
    dt1 = time.perf_counter() - t0
    extra = max(0, int(budget_s / max(dt1, 1e-9)) - 1)
    t0 = time.perf_counter()
    if extra:
        f = ref.step(p, f, extra)
    dt = time.perf_counter() - t0
    steps = extra if extra else 1
    sec = dt if extra else dt1
    assert np.isfinite(f).all()
    # one thread on a 64^3 crop of the same workload, for scale
    c1 = dict(cfg, nx=64, ny=64, nz=64)
    p1 = ref.make_params(c1, nthreads=1)
    rho1, u1 = li.init_fields(c1, dict(init, droplets=[dict(d, center=(32.0, 32.0, 32.0), r0=12.0)
                                                         for d in init["droplets"][:1]]))
    f1 = ref.equilibrium(p1, rho1, u1)
    t0 = time.perf_counter()
    f1 = ref.step(p1, f1, 2)
    st1 = rho1.size * 2 / (time.perf_counter() - t0) / 1e6
    return {"value": N * steps / sec / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"full {cfg['nx']}x{cfg['ny']}x{cfg['nz']} lattice, FP64 dense-matrix oracle, "
                      f"{steps} step(s) after 1 untimed step",
            "single_thread_mlups": round(st1, 3), "single_thread_sample": "64^3 droplet, 2 steps, 1 thread",
            "host_cpu": host_cpu(), "logical_cpus": os.cpu_count()}


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_workloads(threads=16):
    """The oracle's rate (MLUPS, FP64) on the host for each standard
    workload: a few steps each, since the rate is per lattice update; the
    batch is sampled by one step of each of its first 32 runs; one more
    figure with a single thread on the 128^3 lattice."""
    import lbm_inputs as li
    from oracle import ref
    threads = min(threads, os.cpu_count() or 1)
    work = [("droplet_32", li.c1_droplet, 200), ("laplace_128", lambda: li.c2_laplace(24), 10),
            ("two_droplets_256", li.c3_two_droplets, 3), ("sessile_384x384x192", lambda: li.c4_sessile(60.0), 2)]
    out = []
    for name, fn, steps in work:
        cfg, init = fn()
        p = ref.make_params(cfg, nthreads=threads)
        f = ref.equilibrium(p, *li.init_fields(cfg, init))
        t0 = time.perf_counter()
        f = ref.step(p, f, steps)
        n = cfg["nx"] * cfg["ny"] * cfg["nz"]
        out.append({"workload": name, "nodes": n, "oracle_mlups": round(n * steps / (time.perf_counter() - t0) / 1e6, 2),
                    "threads": threads, "steps": steps})
        del f
    t0 = time.perf_counter()
    done = 0
    for pp, init in li.c5_batch()[:32]:
        pr = ref.make_params(pp, nthreads=threads)
        ref.step(pr, ref.equilibrium(pr, *li.init_fields(pp, init)), 1)
        done += pp["nx"] * pp["ny"] * pp["nz"]
    out.append({"workload": "batch_256_runs", "oracle_mlups": round(done / (time.perf_counter() - t0) / 1e6, 2),
                "threads": threads, "sample": "1 step of each of the first 32 runs"})
    cfg, init = li.c2_laplace(24)
    p = ref.make_params(cfg, nthreads=1)
    f = ref.equilibrium(p, *li.init_fields(cfg, init))
    t0 = time.perf_counter()
    ref.step(p, f, 2)
    out.append({"workload": "laplace_128", "oracle_mlups": round(128 ** 3 * 2 / (time.perf_counter() - t0) / 1e6, 3),
                "threads": 1, "steps": 2, "host_cpu": host_cpu(), "logical_cpus": os.cpu_count()})
    return out


def main():
    a = parse()
    if a.cpu_workloads:
        for row in cpu_baseline_workloads():
            print(json.dumps(row), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not implemented (--gpus must be 1)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    if a.copy_probe:
        copy_probe()
        return
    if a.ceiling_probe:
        print(json.dumps(ceiling_probe(storage="f16s" if a.storage in ("f16s", "f16n") else "f32")), flush=True)
        return
    from paper_1805_08643_amd.binding import algorithmic_bytes_per_node

    if a.workload == "batch_256":
        out = {"workload": "batch_256: 256 periodic droplet runs, L ~ U{32, 48, 64, 96}, seed 1805",
               "batch": bench_batch(a.storage, steps=a.steps // 4 or 10)}
        print(json.dumps(out), flush=True)
        return
    tile = tuple(int(v) for v in a.tile.split(",")) if a.tile else None
    lat, cfg, init = make_lattice(a.storage, a.op, a.mode, a.workload, tile)
    mode = lat.mode
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    ms, wall, kms = time_steps(lat, a.steps, a.warmup, kernel_timing=True)
    diag = lat.diagnostics()
    tile = lat.get_tile()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ms_step = ms / a.steps
    mlups = N / (ms_step * 1e-3) / 1e6
    bpn = algorithmic_bytes_per_node(a.storage)
    achieved = bpn * N / (kms * 1e-3) / 1e9
    traffic = read_traffic(a.storage, a.op, mode, a.workload)
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.storage == "f64" else "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {WORKLOADS[a.workload]}",
                   "storage": a.storage, "op": a.op, "nodes": N, "tile": list(tile), "step_mode": mode},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": KERNEL_NAMES.get(mode, KERNEL_NAMES["fused"]),
                     "kernel_ms": round(kms, 5), "algorithmic_bytes_per_node": bpn},
        "mass": diag["mass"], "nonfinite": diag["nonfinite"],
    }
    if not a.no_variants and a.workload == WORKLOAD:
        var = {}
        for st, op, md in [("f32", "nonorth", "fused"), ("f32", "nonorth", "pairs"), ("f32", "nonorth", "split"),
                           ("f16s", "nonorth", "fused"),
                           ("f16s", "nonorth", "pairs"), ("f16s", "nonorth", "quads"), ("f16s", "nonorth", "split"),
                           ("f16n", "nonorth", "split"), ("f32", "orth", None),
                           ("f64", "nonorth", "fused")]:
            key = f"{st}_{op}_{md or 'default'}"
            if (st, op) == (a.storage, a.op) and md in (None, mode):
                var[key] = round(mlups, 1)
                continue
            l2, c2, _ = make_lattice(st, op, md)
            m2, _, k2 = time_steps(l2, max(50, a.steps // 4), 10, kernel_timing=True)
            var[key] = round(N / (m2 / max(50, a.steps // 4) * 1e-3) / 1e6, 1)
            var[f"{key}_hbm_frac"] = round(algorithmic_bytes_per_node(st) * N / (k2 * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
            l2.close()
            del l2
            torch.cuda.empty_cache()
        out["variants_mlups"] = var
        out["batch"] = {st: bench_batch(st) for st in ("f32", "f16s", "f16n")}
        out["precision"] = precision_check()
    cp = ceiling_probe(reps=10, quick=True)["rows"]
    out["roofline"]["copy_probe_GBps"] = cp[0]["GBps_read_plus_write"]
    out["roofline"]["stream19_probe_GBps"] = cp[1]["GBps_read_plus_write"]
    out["roofline"]["probes"] = ("hand-written device copy and 19-plane stream of the FP32 256^3 step's bytes "
                                 "(2.55 GB read + written), streaming stores")
    out["roofline"]["frac_of_copy_probe"] = round(achieved / cp[0]["GBps_read_plus_write"], 4)
    out["roofline"]["frac_of_stream19_probe"] = round(achieved / cp[1]["GBps_read_plus_write"], 4)
    if not a.no_cpu and a.workload == WORKLOAD:
        out["cpu_baseline"] = cpu_baseline(cfg, init, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
