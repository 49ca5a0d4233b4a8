"""The tuning cache on the GPU: a lattice and a batch tuned once are
restored from the JSON file on the next run of the same configuration,
without timing, and step to the same bits."""
import pytest
import torch

import lbm_inputs as li
from paper_1805_08643_amd.binding import Batch, Lattice, f16_exp_for
from paper_1805_08643_amd.tune_cache import TuneCache

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_lattice_tile_restored_from_cache(tmp_path):
    _need_gpu()
    cfg, init = li.c3_two_droplets(n=64)
    cfg = dict(cfg, storage="f16s", rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
    path = str(tmp_path / "tune.json")
    states = []
    for expect_hit in (False, True):
        print(f"[gpu] tune cache lattice, expect hit {expect_hit}", flush=True)
        lat = Lattice(cfg).init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
        cache = TuneCache(path)
        tile, hit = cache.tune_lattice(lat, trials=2)
        assert hit == expect_hit and tuple(lat.get_tile()) == tile
        lat.step(5)
        states.append(lat.save_state().clone())
        lat.close()
    assert torch.equal(states[0], states[1])


def test_batch_tuning_restored_from_cache(tmp_path):
    _need_gpu()
    runs = li.c5_batch(n_runs=6, seed=7, sizes=(32, 48))
    cfgs = [dict(p, storage="f32") for p, _ in runs]
    path = str(tmp_path / "tune.json")
    got = []
    for expect_hit in (False, True):
        print(f"[gpu] tune cache batch, expect hit {expect_hit}", flush=True)
        b = Batch(cfgs)
        for k, (_, init) in enumerate(runs):
            b.init_droplets(k, init["droplets"], init["rho_L"], init["rho_V"], init["W"])
        shape, hit = TuneCache(path).tune_batch(b, trials=1)
        assert hit == expect_hit and b.tuning() == shape
        b.step(4, 2)
        got.append([b.read_populations(k).clone() for k in range(len(runs))])
        b.close()
    assert all(torch.equal(x, y) for x, y in zip(*got))
