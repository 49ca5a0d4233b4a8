"""lbm_step_noalloc, the step for callers that cannot allocate memory, against
lbm_step on a context with the same parameters: the raw states after each
call must be identical bit for bit (the same kernels and launch shape run;
only the scratch of the wall planes lives elsewhere).  Calls follow each
other in one process, each lattice smaller than the one before, so a call
that read the previous call's scratch contents instead of its own would
show."""
import numpy as np
import pytest
import torch

import lbm_inputs as li
from paper_1805_08643_amd import binding
from paper_1805_08643_amd.binding import Lattice, f16_exp_for

pytestmark = pytest.mark.gpu

ELEM = {"f64": 8, "f32": 4, "f16s": 2, "f16n": 2}


def _cases():
    big, big_init = li.c4_sessile(60.0, nx=48, ny=40, nz=20, r0=9.0)
    mid, mid_init = li.c4_sessile(90.0, nx=40, ny=32, nz=16, r0=8.0)
    small, small_init = li.c4_sessile(120.0, nx=24, ny=20, nz=10, r0=5.0)
    per, per_init = li.c3_two_droplets(n=32)
    return [
        ("walls_48x40x20_60deg_f32", dict(big, storage="f32"), big_init, 3),
        ("walls_40x32x16_90deg_f16n", dict(mid, storage="f16n", f16_exp=f16_exp_for(1.25 * mid_init["rho_L"])),
         mid_init, 2),
        ("walls_24x20x10_120deg_f64", dict(small, storage="f64"), small_init, 2),
        ("periodic_32_f16s", dict(per, storage="f16s", rho_ref=per_init["rho_V"],
                                  f16_exp=f16_exp_for(1.25 * per_init["rho_L"])), per_init, 2),
    ]


def _raw(lat, nbytes):
    return lat.save_state()[:nbytes].clone()


def test_noalloc_step_bit_identical_to_context_step():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    for name, cfg, init, steps in _cases():
        print(f"[gpu] noalloc {name}: {steps} calls", flush=True)
        N = cfg["nx"] * cfg["ny"] * cfg["nz"]
        nbytes = binding.population_bytes(cfg["storage"], N)
        ref_lat = Lattice(cfg)
        ref_lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
        src = _raw(ref_lat, nbytes)
        dst = torch.empty_like(src)
        assert src.data_ptr() % 256 == 0 and dst.data_ptr() % 256 == 0
        p = binding.make_params(cfg)
        stream = torch.cuda.current_stream(dev).cuda_stream
        for k in range(steps):
            binding.lbm_step_noalloc(p, src.data_ptr(), dst.data_ptr(), stream)
            ref_lat.step(1)
            torch.cuda.synchronize(dev)
            want = _raw(ref_lat, nbytes)
            same = torch.equal(dst, want)
            print(f"  call {k + 1}: bit-identical {same}", flush=True)
            assert same, (name, k)
            src, dst = dst, src
        ref_lat.close()


def test_noalloc_step_rejects_oversized_wall_planes_and_bad_buffers():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # Every call below is rejected before any HIP call, so the small buffers
    # are never touched.
    p = binding.make_params(li.params(2048, 2048, 2, storage="f64", wall_z=1, theta_wall_deg=60.0))
    buf = torch.empty(256, dtype=torch.uint8, device="cuda:0")
    buf2 = torch.empty(256, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(binding.LbmError) as e:
        binding.lbm_step_noalloc(p, buf.data_ptr(), buf2.data_ptr(), 0)
    assert e.value.status == -5 and "scratch" in str(e.value)
    small = binding.make_params(li.params(8, 8, 8, storage="f32"))
    with pytest.raises(binding.LbmError) as e:
        binding.lbm_step_noalloc(small, buf.data_ptr(), buf.data_ptr(), 0)
    assert e.value.status == -1
    with pytest.raises(binding.LbmError) as e:
        binding.lbm_step_noalloc(small, buf.data_ptr() + 8, buf2.data_ptr(), 0)
    assert e.value.status == -1
