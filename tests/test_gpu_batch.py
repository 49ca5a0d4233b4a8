"""Batched runs: one persistent launch per step over many independent
lattices of uneven size, plain and hipGraph-replayed, against the oracle and
against single-lattice launches."""
import numpy as np
import pytest
import torch

import lbm_inputs as li
from oracle import ref
from paper_1805_08643_amd import binding
from paper_1805_08643_amd.binding import Lattice

pytestmark = pytest.mark.gpu


class Batch(binding.Batch):
    def pops(self, k):
        return self.read_populations(k).cpu().numpy()


def _runs(storage, sizes=(12, 16, 20, 24, 18), seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for L in sizes:
        t = float(rng.uniform(0.6, 0.9))
        tau = float(rng.uniform(0.6, 1.2))
        a, W = li.interface_recipe(t)
        p = li.params(L, L, L, T_over_Tc=t, tau_nu=tau, storage=storage, eos_a=a)
        rl, rv = li.coexistence(t)
        p["rho_ref"] = rv
        p["f16_exp"] = binding.f16_exp_for(1.25 * rl)
        init = dict(droplets=[dict(center=(L / 2, L / 2, L / 2), r0=0.25 * L)], rho_L=rl, rho_V=rv, W=W)
        out.append((p, init))
    return out


@pytest.mark.parametrize("graph_steps", [0, 2, 3])
def test_batch_fp64_matches_oracle(graph_steps):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs("f64")
    print(f"[gpu] batch f64 runs={[r[0]['nx'] for r in runs]} graph_steps={graph_steps}", flush=True)
    b = Batch([r[0] for r in runs])
    fields = [li.init_fields(p, i) for p, i in runs]
    for k, (rho, u) in enumerate(fields):
        b.init_fields(k, rho, u)
    b.step(6, graph_steps)
    for k, (p, _) in enumerate(runs):
        got = b.pops(k)
        op = ref.make_params(p)
        want = ref.step(op, ref.equilibrium(op, *fields[k]), 6)
        e = float((np.abs(got - want) / want.sum(0)[None]).max())
        print(f"  run {k} L={p['nx']}: err {e:.3e}")
        assert e < 1e-12
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16s", "f16n"])
def test_batch_bit_identical_to_single_lattices(storage):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs(storage, sizes=(32, 48, 20, 36))
    b = Batch([r[0] for r in runs])
    for k, (p, init) in enumerate(runs):
        b.init_fields(k, *li.init_fields(p, init))
    b.step(5, 4)  # one 4-step graph replay + one plain launch
    for k, (p, init) in enumerate(runs):
        lat = Lattice(p)
        lat.init_fields(*li.init_fields(p, init)).step(5)
        assert np.array_equal(b.pops(k), lat.read_populations().cpu().numpy()), k
        lat.close()
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_batch_step_modes_bit_identical(storage):
    """Two nodes per thread, one node per thread and the split step (the
    default where it applies) give the same populations in a batch."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs(storage, sizes=(32, 48, 20, 36))
    out = {}
    for mode in ("pairs", "fused", "split"):
        b = Batch([r[0] for r in runs])
        assert b.step_mode() == "split"
        b.set_step_mode(mode)
        assert b.step_mode() == mode
        for k, (p, init) in enumerate(runs):
            b.init_fields(k, *li.init_fields(p, init))
        b.step(5, 4)
        out[mode] = [b.pops(k) for k in range(len(runs))]
        b.close()
    for k in range(len(runs)):
        assert np.array_equal(out["pairs"][k], out["fused"][k]), k
        assert np.array_equal(out["pairs"][k], out["split"][k]), k


@pytest.mark.parametrize("storage", ["f32", "f16s", "f16n"])
def test_batch_split_wide_run(storage):
    """A run 132 nodes wide takes 128-wide split tiles, whose halo ring is
    larger than the pulling waves: the batch launches the variant in which
    colliding waves take the rest of the ring, also for the small runs."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs(storage, sizes=(20, 24))
    p, init = runs[0]
    wide = dict(p, nx=132, ny=12, nz=10)
    init = dict(init, droplets=[dict(center=(66, 6, 5), r0=4.0)])
    runs = [(wide, init)] + runs
    print(f"[gpu] batch split wide {storage} runs={[(r[0]['nx'], r[0]['ny'], r[0]['nz']) for r in runs]}", flush=True)
    b = Batch([r[0] for r in runs])
    b.set_step_mode("split")
    for k, (q, i) in enumerate(runs):
        b.init_fields(k, *li.init_fields(q, i))
    b.step(4, 3)
    for k, (q, i) in enumerate(runs):
        lat = Lattice(q)
        if storage != "f16n":  # F16N has the split step only
            lat.set_step_mode("fused")
        lat.init_fields(*li.init_fields(q, i)).step(4)
        got = b.pops(k)
        assert np.isfinite(got).all(), k
        assert np.array_equal(got, lat.read_populations().cpu().numpy()), k
        lat.close()
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16s", "f16n"])
def test_batch_split_store_policies_bit_identical(storage):
    """Non-temporal and cached population stores give the same bits in a
    batch, in plain launches and graph replays."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs(storage, sizes=(32, 48, 20, 36))
    out = {}
    for policy in ("cached", "stream"):
        b = Batch([r[0] for r in runs])
        b.set_step_mode("split").set_store_policy(policy)
        for k, (p, init) in enumerate(runs):
            b.init_fields(k, *li.init_fields(p, init))
        b.step(5, 2)
        out[policy] = [b.pops(k) for k in range(len(runs))]
        b.close()
    for k in range(len(runs)):
        assert np.array_equal(out["cached"][k], out["stream"][k]), k


def test_batch_split_rejects_unsuitable_runs():
    """F16S split needs nx % 4 == 0 in every run; an F16N batch runs the
    split step only."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs("f16s", sizes=(32, 18))
    b = Batch([r[0] for r in runs])
    with pytest.raises(binding.LbmError) as e:
        b.set_step_mode("split")
    assert e.value.status == -5
    assert b.step_mode() == "pairs"
    b.close()
    fn = Batch([r[0] for r in _runs("f16n", sizes=(32, 20))])
    assert fn.step_mode() == "split"
    with pytest.raises(binding.LbmError) as e:
        fn.set_step_mode("fused")
    assert e.value.status == -5 and fn.step_mode() == "split"
    fn.close()


def test_batch_full_workload_sampled_runs():
    """The 256-run workload (L in {32, 48, 64, 96}), FP32: eight runs checked
    against the oracle after 3 steps."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = li.c5_batch()
    cfgs = [dict(p, storage="f32") for p, _ in runs]
    b = Batch(cfgs)
    for k, (p, init) in enumerate(runs):
        b.init_droplets(k, init["droplets"], init["rho_L"], init["rho_V"], init["W"])
    b.step(3, 3)
    for k in [0, 1, 7, 64, 100, 128, 200, 255]:
        p, init = runs[k]
        got = b.pops(k)
        op = ref.make_params(p)
        want = ref.step(op, ref.equilibrium(op, *li.init_fields(p, init)), 3)
        e = float((np.abs(got - want) / want.sum(0)[None]).max())
        print(f"  run {k} L={p['nx']}: err {e:.3e}")
        assert e < 1.5e-5
    b.close()


def test_batch_full_workload_100_steps_split():
    """The spot check of the 256-run workload: eight runs of every size, FP32,
    in the split step that the tuned batch uses, against the oracle after 100
    steps (ten 10-step graph replays), within the stated FP32 bound of 1e-5
    relative to the density."""
    import os
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = li.c5_batch()
    cfgs = [dict(p, storage="f32") for p, _ in runs]
    b = Batch(cfgs)
    b.set_step_mode("split")
    for k, (p, init) in enumerate(runs):
        b.init_droplets(k, init["droplets"], init["rho_L"], init["rho_V"], init["W"])
    b.step(100, 10)
    threads = min(16, os.cpu_count() or 1)
    for k in [0, 1, 7, 64, 100, 128, 200, 255]:
        p, init = runs[k]
        got = b.pops(k)
        op = ref.make_params(p, nthreads=threads)
        want = ref.step(op, ref.equilibrium(op, *li.init_fields(p, init)), 100)
        e = float((np.abs(got - want) / want.sum(0)[None]).max())
        print(f"  run {k} L={p['nx']}: err {e:.3e} after 100 steps", flush=True)
        assert np.isfinite(got).all()
        assert e < 1e-5
    b.close()


def test_batch_variable_viscosity_matches_single_lattices():
    """Per-run parameters travel through the batch descriptor, including the
    density-dependent viscosity."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs("f32", sizes=(24, 32, 20))
    cfgs = []
    for k, (p, init) in enumerate(runs):
        cfgs.append(dict(p, nu_ratio=float(2 + 3 * k), visc_rho_L=init["rho_L"], visc_rho_V=init["rho_V"]))
    b = Batch(cfgs)
    for k, (p, init) in enumerate(runs):
        b.init_fields(k, *li.init_fields(cfgs[k], init))
    b.step(4, 2)
    for k, (p, init) in enumerate(runs):
        lat = Lattice(cfgs[k])
        lat.init_fields(*li.init_fields(cfgs[k], init)).step(4)
        assert np.array_equal(b.pops(k), lat.read_populations().cpu().numpy()), k
        lat.close()
    b.close()


def test_batch_diagnostics_and_status_per_run():
    """Per-run diagnostics equal those of the same lattice run alone (same
    populations, same fixed-order reduction), and a run whose populations are
    not finite is flagged alone.  The NaN is planted in that run's initial
    density from the host; NaN arithmetic raises nothing on the device."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = _runs("f32", sizes=(20, 24, 16))
    b = Batch([r[0] for r in runs])
    fields = [li.init_fields(p, i) for p, i in runs]
    rho_bad = np.array(fields[1][0], copy=True)
    rho_bad.reshape(-1)[7] = np.nan
    print(f"[gpu] batch status runs={[r[0]['nx'] for r in runs]} nan in run 1", flush=True)
    for k, (rho, u) in enumerate(fields):
        b.init_fields(k, rho_bad if k == 1 else rho, u)
    b.step(3, 0)
    assert b.runs == 3
    assert b.status() == [0, -4, 0]
    for k in (0, 2):
        p, init = runs[k]
        lat = Lattice(p)
        lat.init_fields(*fields[k]).step(3)
        c = (p["nx"] / 2, p["ny"] / 2, p["nz"] / 2)
        want = lat.diagnostics(c, 3.0, 7.0)
        got = b.diagnostics(k, c, 3.0, 7.0)
        lat.close()
        assert got["status"] == 0 and got["nonfinite"] == 0 and got["step"] == 3
        for key in ("mass", "momentum", "max_u", "p_in", "p_out", "rho_in", "rho_out", "n_in", "n_out"):
            assert got[key] == want[key], key
    bad = b.diagnostics(1)
    assert bad["status"] == -4 and bad["nonfinite"] > 0
    assert "run 1" in binding.lbm_last_error()
    b.close()


def test_batch_flags_the_diverging_run_only():
    """Three FP64 runs, the middle one unstable (T = 0.5 T_c, s_nu = 1.9):
    after 100 steps only that run reports non-finite populations."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    runs = [li.cold_droplet(1.0), li.cold_droplet(1.9), li.cold_droplet(1.0, n=20, T_over_Tc=0.6)]
    print("[gpu] batch divergence runs s_nu=(1.0, 1.9, 1.0)", flush=True)
    b = Batch([r[0] for r in runs])
    for k, (p, init) in enumerate(runs):
        b.init_fields(k, *li.init_fields(p, init))
    b.step(100, 25)
    assert b.status() == [0, -4, 0]
    b.close()
