"""GPU parity: the HIP library, called through the C ABI, against the FP64
oracle on the same seeded inputs.

Error measure: for populations, max over nodes x and directions a of
|f_gpu - f_oracle| / rho_oracle(x) (density-normalised absolute error; a
population is at most rho and near-zero populations have no meaningful
relative error).  Tolerances:
  * FP64 storage and arithmetic: 1e-12 (stated bound for FP64 runs).
  * FP32: one step rounds every population once on store (2^-24 relative)
    and the collision forms moment differences of O(rho) size, ~30 roundings
    deep: ~30 * 6e-8 = 2e-6 per step; bound 5e-6 per step, capped at the
    stated FP32 bound of 1e-5 relative to the density (``fp32_bound``).
  * Shifted FP16 storage: tests/test_gpu_f16s.py, with bounds from the
    format itself.
"""
import numpy as np
import pytest
import torch

import lbm_inputs as li
from oracle import ref
from paper_1805_08643_amd import binding, tuning
from paper_1805_08643_amd.binding import Lattice, f16_exp_for

pytestmark = pytest.mark.gpu

Q = 19


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_states(cfg, rho, u, checkpoints, tile=None, mode=None):
    """States after each checkpoint; mode None keeps the library's default
    step kernel (the split step where it applies, else two nodes per thread,
    else one)."""
    _need_gpu()
    print(f"[gpu] {cfg['nx']}x{cfg['ny']}x{cfg['nz']} op={cfg.get('op')} storage={cfg.get('storage')} "
          f"wall={cfg.get('wall_z', 0)} tile={tile} mode={mode} steps={checkpoints}", flush=True)
    lat = Lattice(cfg)
    if mode is not None:
        lat.set_step_mode(mode)
    if tile is not None:
        lat.set_tile(*tile)
    lat.init_fields(rho, u)
    out, done = [], 0
    for s in checkpoints:
        lat.step(s - done)
        done = s
        out.append(lat.read_populations().cpu().numpy())
    lat.close()
    return out


def oracle_states(cfg, rho, u, checkpoints):
    p = ref.make_params(cfg)
    f = ref.equilibrium(p, rho, u)
    out, done = [], 0
    for s in checkpoints:
        f = ref.step(p, f, s - done)
        done = s
        out.append(f)
    return out


W_CLASS = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def fp32_bound(steps):
    """FP32 storage and arithmetic: 5e-6 per step, capped at 1e-5."""
    return min(5e-6 * steps, 1e-5)


def rho_err(got, want):
    rho = want.sum(0)
    return float((np.abs(got - want) / rho[None, :]).max())


CASES = {
    # name: (cfg, init, tile)
    "droplet_32": lambda op: (*li.c1_droplet(op=op), (32, 8, 8)),
    "ragged_70x37x21": lambda op: (dict(li.c3_two_droplets(n=64, op=op)[0], nx=70, ny=37, nz=21),
                                   dict(li.c3_two_droplets(n=64)[1]), (32, 8, 8)),
    "ragged_68x37x21": lambda op: (dict(li.c3_two_droplets(n=64, op=op)[0], nx=68, ny=37, nz=21),
                                   dict(li.c3_two_droplets(n=64)[1]), (32, 8, 8)),
    "walls_40x33x19_60deg": lambda op: (*li.c4_sessile(60.0, nx=40, ny=33, nz=19, r0=8.0), (16, 8, 7)),
    "walls_37x20x12_120deg": lambda op: (*li.c4_sessile(120.0, nx=37, ny=20, nz=12, r0=6.0), (32, 4, 5)),
    # density-dependent viscosity: nu_L = 0.01 in the liquid, nu_V = 10 nu_L
    "visc_two_droplets_48": lambda op: (
        dict(li.c3_two_droplets(n=48, op=op)[0], tau_nu=0.53, nu_ratio=10.0,
             visc_rho_L=li.coexistence(0.6)[0], visc_rho_V=li.coexistence(0.6)[1]),
        li.c3_two_droplets(n=48)[1], (16, 8, 12)),
}


def _case(name, op, storage):
    cfg, init, tile = CASES[name](op)
    cfg = dict(cfg, op=op, storage=storage)
    if storage == "f16s":
        cfg["rho_ref"] = init["rho_V"]
        cfg["f16_exp"] = f16_exp_for(1.25 * init["rho_L"])
    if name.startswith("ragged"):
        # droplets placed for a 64^3 box; shift into the ragged box
        init = dict(init, droplets=[dict(d, center=(d["center"][0] + 3, d["center"][1] - 14, d["center"][2] - 22))
                                    for d in init["droplets"]])
    rho, u = li.init_fields(cfg, init)
    return cfg, rho, u, tile


@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("name", list(CASES))
def test_fp64_parity(name, op):
    cfg, rho, u, tile = _case(name, op, "f64")
    cps = [0, 1, 5] if name != "droplet_32" else [0, 1, 10, 100]
    got = gpu_states(cfg, rho, u, cps, tile)
    want = oracle_states(cfg, rho, u, cps)
    for s, g, w in zip(cps, got, want):
        e = rho_err(g, w)
        print(f"  step {s}: err {e:.3e}")
        assert e < 1e-12, (s, e)


def test_fp64_parity_500_steps_droplet_32():
    """The 32^3 stationary droplet at steps 1, 10, 100, 500."""
    cfg, rho, u, tile = _case("droplet_32", "nonorth", "f64")
    cps = [1, 10, 100, 500]
    got = gpu_states(cfg, rho, u, cps, tile)
    want = oracle_states(cfg, rho, u, cps)
    for s, g, w in zip(cps, got, want):
        e = rho_err(g, w)
        print(f"  step {s}: err {e:.3e}")
        assert e < 1e-12, (s, e)


@pytest.mark.parametrize("mode", ["fused", "pairs", "split"])
@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("name", ["droplet_32", "ragged_70x37x21", "walls_40x33x19_60deg", "visc_two_droplets_48"])
def test_fp32_parity(name, op, mode):
    cfg, rho, u, tile = _case(name, op, "f32")
    cps = [1, 10]
    got = gpu_states(cfg, rho, u, cps, tile, mode)
    want = oracle_states(cfg, rho, u, cps)
    for s, g, w in zip(cps, got, want):
        e = rho_err(g, w)
        print(f"  step {s}: err {e:.3e} (bound {fp32_bound(s):.1e})")
        assert e < fp32_bound(s), (s, e)


@pytest.mark.parametrize("mode", ["pairs", "split"])
def test_fp32_density_500_steps_droplet_32(mode):
    """The 32^3 droplet in FP32 storage and arithmetic: the density field after
    500 steps within 1e-5 of the FP64 oracle, relative to the local density."""
    cfg, rho, u, tile = _case("droplet_32", "nonorth", "f32")
    got = gpu_states(cfg, rho, u, [500], None, mode)[0]
    want = oracle_states(cfg, rho, u, [500])[0]
    rg, rw = got.sum(0), want.sum(0)
    e = float((np.abs(rg - rw) / rw).max())
    print(f"  500 steps: density err {e:.3e}")
    assert e < 1e-5


def test_f16_storage_format_round_trip():
    """Populations written through the C ABI and read back equal the stated
    format exactly: v = fbar rounded to FP32, h = (v - w rho_ref) 2^e
    evaluated exactly and rounded once (nearest even) to binary16; reading
    gives h 2^-e + w rho_ref rounded once to FP32."""
    _need_gpu()
    cfg, init = li.c3_two_droplets(n=24)
    cfg = dict(cfg, storage="f16s", rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
    rho, u = li.init_fields(cfg, init)
    f = ref.equilibrium(ref.make_params(cfg), rho, u) * (1 + 0.05 * li.random_populations(24, 24, 24, 9, -1, 1))
    lat = Lattice(cfg)
    lat.write_populations(f)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    hs = 2.0 ** cfg["f16_exp"]
    shift = (W_CLASS * cfg["rho_ref"]).astype(np.float32).astype(np.float64)[:, None]
    v = f.astype(np.float32).astype(np.float64)
    h16 = ((v - shift) * hs).astype(np.float16)  # exact in FP64, one rounding to binary16
    want = (h16.astype(np.float64) / hs + shift).astype(np.float32).astype(np.float64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("mode", ["fused", "pairs"])
def test_tiles_give_bit_identical_results(mode):
    """Every node's arithmetic is independent of the tiling, so any tile
    shape (including ragged tails) must give the same bits."""
    cfg, rho, u, _ = _case("ragged_70x37x21", "nonorth", "f32")
    ref_state = None
    for tile in [(32, 8, 8), (64, 4, 21), (16, 16, 3), (70, 4, 5), (8, 32, 1), (128, 8, 21)]:
        if mode == "fused" and tile[0] * tile[1] > 512:
            continue
        s = gpu_states(cfg, rho, u, [3], tile, mode)[0]
        if ref_state is None:
            ref_state = s
        else:
            assert np.array_equal(s, ref_state), tile


@pytest.mark.parametrize("name,storage", [("ragged_70x37x21", "f32"), ("walls_37x20x12_120deg", "f32"),
                                          ("walls_40x33x19_60deg", "f64"), ("droplet_32", "f16s")])
@pytest.mark.parametrize("slab", [1, 5, 64])
def test_slab_mode_bit_identical_to_fused(name, storage, slab):
    """The two-pass slab step computes every node with the same arithmetic as
    the fused kernel, so the populations agree bit for bit."""
    cfg, rho, u, tile = _case(name, "nonorth", storage)
    fused = gpu_states(cfg, rho, u, [3], tile, "fused")[0]
    lat = Lattice(cfg)
    lat.set_step_mode("slabs", slab)
    lat.init_fields(rho, u).step(3)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


PAIR_CASES = [("ragged_70x37x21", "f32", (64, 8, 5)), ("ragged_70x37x21", "f16s", (32, 4, 7)),
              ("walls_40x33x19_60deg", "f32", (16, 8, 7)), ("walls_40x33x19_60deg", "f16s", (40, 2, 19)),
              ("droplet_32", "f32", (2, 16, 4)), ("droplet_32", "f16s", (32, 8, 8))]


@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("name,storage,tile", PAIR_CASES)
def test_pair_mode_bit_identical_to_fused(name, storage, tile, op):
    """Two nodes per thread with wide accesses: same arithmetic per node as
    the one-node kernel, so the same populations bit for bit.  The tiles
    cover ragged last tiles in x and y (a pair starting at nx supplies the
    wrapped columns), seam lanes at both ends of x, and walls."""
    cfg, rho, u, ftile = _case(name, op, storage)
    fused = gpu_states(cfg, rho, u, [3], ftile, "fused")[0]
    print(f"[gpu] pairs {name} {storage} {op} tile={tile}", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode("pairs").set_tile(*tile)
    lat.init_fields(rho, u).step(3)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_pair_mode_two_column_lattice(storage):
    """nx = 2: one pair per row, on the seam at both ends."""
    cfg = li.params(2, 6, 5, T_over_Tc=0.8, storage=storage, rho_ref=0.02, f16_exp=f16_exp_for(0.4))
    rho, u = li.random_fields(2, 6, 5, seed=11)
    fused = gpu_states(cfg, rho, u, [2], (2, 6, 5), "fused")[0]
    lat = Lattice(cfg)
    lat.set_step_mode("pairs").set_tile(2, 6, 5)
    lat.init_fields(rho, u).step(2)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


def test_default_step_mode():
    _need_gpu()
    for shape, storage, want in [((32, 8, 8), "f32", "split"), ((32, 8, 8), "f16s", "split"),
                                 ((34, 8, 8), "f16s", "pairs"), ((32, 8, 8), "f64", "fused"),
                                 ((33, 8, 8), "f32", "fused")]:
        lat = Lattice(li.params(*shape, storage=storage))
        assert lat.step_mode() == want, (shape, storage)
        lat.close()


def test_pair_mode_rejections():
    _need_gpu()
    lat = Lattice(li.params(32, 8, 8, storage="f64"))
    with pytest.raises(binding.LbmError) as e:
        lat.set_step_mode("pairs")
    assert e.value.status == -5
    lat.close()
    lat = Lattice(li.params(33, 8, 8, storage="f32"))
    with pytest.raises(binding.LbmError) as e:
        lat.set_step_mode("pairs")
    assert e.value.status == -5
    lat.close()
    lat = Lattice(li.params(32, 8, 8, storage="f32"))
    lat.set_step_mode("pairs")
    with pytest.raises(binding.LbmError) as e:
        lat.set_tile(15, 4, 4)
    assert e.value.status == -1
    lat.close()


# Four nodes per thread (F16S): ragged tiles in x and y (with the wrap quad
# that starts at nx), seam lanes at both ends, walls, a lattice one quad wide.
QUAD_CASES = [("ragged_68x37x21", (32, 4, 7)), ("ragged_68x37x21", (68, 8, 21)), ("walls_40x33x19_60deg", (40, 4, 7)),
              ("droplet_32", (32, 16, 8)), ("visc_two_droplets_48", (16, 8, 12))]


@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("name,tile", QUAD_CASES)
def test_quad_mode_bit_identical_to_fused(name, tile, op):
    cfg, rho, u, ftile = _case(name, op, "f16s")
    fused = gpu_states(cfg, rho, u, [3], ftile, "fused")[0]
    print(f"[gpu] quads {name} f16s {op} tile={tile}", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode("quads").set_tile(*tile)
    lat.init_fields(rho, u).step(3)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


SPLIT_CASES = [("f16s", "ragged_68x37x21", (32, 4, 7)), ("f16s", "ragged_68x37x21", (68, 8, 21)),
               ("f16s", "walls_40x33x19_60deg", (40, 4, 7)), ("f16s", "droplet_32", (32, 8, 8)),
               ("f16s", "visc_two_droplets_48", (16, 8, 12)),
               ("f32", "ragged_70x37x21", (32, 4, 7)), ("f32", "ragged_70x37x21", (70, 2, 21)),
               ("f32", "walls_40x33x19_60deg", (40, 4, 7)), ("f32", "droplet_32", (32, 8, 8)),
               ("f32", "visc_two_droplets_48", (16, 8, 12))]


@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("storage,name,tile", SPLIT_CASES)
def test_split_mode_bit_identical_to_fused(storage, name, tile, op):
    """Pullers three planes ahead of colliders, planes handed over in LDS:
    the same populations as the one-node kernel."""
    cfg, rho, u, ftile = _case(name, op, storage)
    fused = gpu_states(cfg, rho, u, [3], ftile, "fused")[0]
    print(f"[gpu] split {name} {storage} {op} tile={tile}", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode("split").set_tile(*tile)
    lat.init_fields(rho, u).step(3)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


# Tiles whose halo ring has more nodes than the pulling waves have threads:
# the colliding waves take the rest.  (storage, lattice, tile, walls)
SPLIT_RING_CASES = [("f16s", (132, 21, 9), (128, 8, 9), 0),  # 276-node ring, 20 on a colliding wave
                    ("f32", (132, 13, 9), (128, 4, 9), 1),   # 268, walls in z
                    ("f16s", (8, 210, 6), (4, 200, 6), 1),   # 412
                    ("f32", (6, 260, 5), (2, 252, 5), 0),    # 512: one node for every thread of the block
                    ("f32", (264, 6, 5), (256, 2, 5), 0),    # 520: a second round on one colliding wave
                    ("f32", (260, 9, 5), (256, 2, 5), 1)]    # 520, walls in z


@pytest.mark.parametrize("storage,shape,tile,walls", SPLIT_RING_CASES)
def test_split_mode_halo_ring_beyond_pullers(storage, shape, tile, walls):
    kw = dict(T_over_Tc=0.8, storage=storage, wall_z=walls)
    if walls:
        kw["theta_wall_deg"] = 60.0
    if storage == "f16s":
        kw.update(rho_ref=0.02, f16_exp=f16_exp_for(0.4))
    cfg = li.params(*shape, **kw)
    # A narrow density range keeps the Eq. (57) ghost layer below the C-S
    # singularity at rho = 4 / b, so psi stays finite at the walls.
    rho, u = li.random_fields(*shape, seed=17, rho_lo=0.15, rho_hi=0.25)
    fused = gpu_states(cfg, rho, u, [3], (min(shape[0], 32), 4, shape[2]), "fused")[0]
    assert np.isfinite(fused).all()
    print(f"[gpu] split ring {storage} {shape} tile={tile} walls={walls}", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode("split").set_tile(*tile)
    lat.init_fields(rho, u).step(3)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


@pytest.mark.parametrize("mode", ["fused", "slabs"])
def test_mode_switch_replaces_a_tile_the_new_mode_cannot_run(mode):
    """An FP32 lattice 132 wide in pair mode with a 128 x 8 tile: one node per
    thread that tile would need 1024 threads, so switching mode picks a tile
    the one-node kernel can run, bit-identical to a stated one."""
    cfg = li.params(132, 12, 10, T_over_Tc=0.8, storage="f32")
    rho, u = li.random_fields(132, 12, 10, seed=21, rho_lo=0.15, rho_hi=0.25)
    want = gpu_states(cfg, rho, u, [2], (32, 4, 10), "fused")[0]
    print(f"[gpu] mode switch pairs -> {mode} on 132x12x10", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode("pairs")
    lat.set_tile(128, 8, 10)
    t0 = lat.get_tile()
    lat.set_step_mode(mode)
    t1 = lat.get_tile()
    assert t0[0] * t0[1] > 512 and t1[0] * t1[1] <= 512, (t0, t1)
    lat.init_fields(rho, u).step(2)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("storage,name,tile", [("f16s", "droplet_32", (32, 8, 8)),
                                               ("f32", "walls_40x33x19_60deg", (40, 4, 7)),
                                               ("f32", "ragged_70x37x21", (70, 2, 21))])
def test_split_store_policies_bit_identical(storage, name, tile):
    """Non-temporal and cached population stores give the same bits."""
    cfg, rho, u, _ = _case(name, "nonorth", storage)
    out = {}
    for policy in ("cached", "stream"):
        print(f"[gpu] split {name} {storage} stores={policy}", flush=True)
        lat = Lattice(cfg)
        lat.set_step_mode("split").set_store_policy(policy)
        lat.set_tile(*tile)
        lat.init_fields(rho, u).step(3)
        out[policy] = lat.read_populations().cpu().numpy()
        lat.close()
    assert np.array_equal(out["cached"], out["stream"])
    lat = Lattice(cfg)
    lat.set_store_policy("auto")
    with pytest.raises(binding.LbmError) as e:
        binding._call("lbm_set_store_policy", binding._vp(lat.ctx), 7)
    assert e.value.status == -1
    lat.close()


def test_split_mode_two_column_lattice():
    """FP32, nx = 2: one group per row, on the seam at both ends at once."""
    cfg = li.params(2, 6, 5, T_over_Tc=0.8, storage="f32")
    rho, u = li.random_fields(2, 6, 5, seed=13)
    fused = gpu_states(cfg, rho, u, [2], (2, 6, 5), "fused")[0]
    lat = Lattice(cfg)
    lat.set_step_mode("split").set_tile(2, 6, 5)
    lat.init_fields(rho, u).step(2)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


def test_split_mode_rejections():
    _need_gpu()
    for shape, storage in [((32, 8, 8), "f64"), ((33, 8, 8), "f32"), ((34, 8, 8), "f16s")]:
        lat = Lattice(li.params(*shape, storage=storage))
        with pytest.raises(binding.LbmError) as e:
            lat.set_step_mode("split")
        assert e.value.status == -5, (shape, storage)
        lat.close()
    lat = Lattice(li.params(32, 32, 8, storage="f16s"))
    lat.set_step_mode("split")
    lat.set_tile(32, 32, 4)  # 256 groups of four: the LDS limit
    # (256, 1): F16S halo rings may take two rounds of 256 threads, not 518 nodes
    for tile in [(30, 4, 4), (32, 40, 4), (128, 9, 4), (256, 1, 4), (260, 1, 4)]:
        with pytest.raises(binding.LbmError) as e:
            lat.set_tile(*tile)
        assert e.value.status == -1, tile
    lat.close()
    # FP32 groups of two: the tallest and the widest tiles of 256 groups are
    # accepted (halo rings of 520 nodes, three rounds); wider, or more
    # groups, are not.
    lat = Lattice(li.params(6, 260, 8, storage="f32"))
    lat.set_step_mode("split")
    lat.set_tile(2, 256, 4)
    lat.set_tile(256, 2, 4)
    for tile in [(258, 2, 4), (2, 257, 4), (256, 3, 4)]:
        with pytest.raises(binding.LbmError) as e:
            lat.set_tile(*tile)
        assert e.value.status == -1, tile
    lat.close()


def test_quad_mode_one_quad_wide_lattice():
    """nx = 4: one quad per row, on the seam at both ends at once."""
    cfg = li.params(4, 6, 5, T_over_Tc=0.8, storage="f16s", rho_ref=0.02, f16_exp=f16_exp_for(0.4))
    rho, u = li.random_fields(4, 6, 5, seed=12)
    fused = gpu_states(cfg, rho, u, [2], (4, 6, 5), "fused")[0]
    lat = Lattice(cfg)
    lat.set_step_mode("quads").set_tile(4, 6, 5)
    lat.init_fields(rho, u).step(2)
    got = lat.read_populations().cpu().numpy()
    lat.close()
    assert np.array_equal(got, fused)


def test_quad_mode_rejections():
    _need_gpu()
    for shape, storage in [((32, 8, 8), "f32"), ((32, 8, 8), "f64"), ((34, 8, 8), "f16s")]:
        lat = Lattice(li.params(*shape, storage=storage))
        with pytest.raises(binding.LbmError) as e:
            lat.set_step_mode("quads")
        assert e.value.status == -5, (shape, storage)
        lat.close()
    lat = Lattice(li.params(32, 8, 8, storage="f16s"))
    lat.set_step_mode("quads")
    with pytest.raises(binding.LbmError) as e:
        lat.set_tile(30, 4, 4)
    assert e.value.status == -1
    lat.close()


def test_init_droplets_on_device_matches_generator():
    _need_gpu()
    cfg, init = li.c3_two_droplets(n=48)
    cfg = dict(cfg, storage="f64")
    rho, u = li.init_fields(cfg, init)
    lat = Lattice(cfg)
    lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
    got = lat.read_populations().cpu().numpy()
    lat.close()
    want = ref.equilibrium(ref.make_params(cfg), rho, u)
    assert rho_err(got, want) < 1e-13


def test_read_fields_and_diagnostics_match_oracle():
    cfg, rho, u, tile = _case("walls_40x33x19_60deg", "nonorth", "f64")
    _need_gpu()
    lat = Lattice(cfg)
    lat.set_tile(*tile)
    lat.init_fields(rho, u).step(4)
    fl = {k: v.cpu().numpy() for k, v in lat.read_fields().items()}
    c = (20.0, 16.5, 8.0)
    d = lat.diagnostics(center=c, r_in=4.0, r_out=12.0)
    lat.close()
    p = ref.make_params(cfg)
    f = ref.step(p, ref.equilibrium(p, rho, u), 4)
    o = ref.fields(p, f)
    for k in ("rho", "p"):
        assert np.abs(fl[k] - o[k]).max() < 1e-12 * np.abs(o[k]).max(), k
    assert np.abs(fl["u"] - o["u"]).max() < 1e-12
    assert abs(d["mass"] - o["rho"].sum()) < 1e-12 * o["rho"].sum()
    mom = (np.array(ref.moments.VELOCITIES).T.astype(float) @ f).sum(1) + 0.5 * o["F"].sum(1)
    assert np.allclose(d["momentum"], mom, rtol=1e-10, atol=1e-13)
    assert abs(d["max_u"] - np.sqrt((o["u"] ** 2).sum(0)).max()) < 1e-12
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dx = np.remainder(x - c[0] + nx / 2, nx) - nx / 2
    dy = np.remainder(y - c[1] + ny / 2, ny) - ny / 2
    dz = z - c[2]
    r2 = (dx * dx + dy * dy + dz * dz).ravel()
    inside, outside = r2 < 16.0, r2 > 144.0
    assert d["n_in"] == inside.sum() and d["n_out"] == outside.sum()
    assert abs(d["p_in"] - o["p"][inside].sum()) < 1e-12 * abs(o["p"][inside].sum())
    assert abs(d["rho_out"] - o["rho"][outside].sum()) < 1e-12 * o["rho"][outside].sum()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_mass_conservation(storage):
    _need_gpu()
    cfg, init = li.c3_two_droplets(n=64)
    cfg = dict(cfg, storage=storage)
    lat = Lattice(cfg)
    lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
    m0 = lat.diagnostics()["mass"]
    lat.step(200)
    d = lat.diagnostics()
    lat.close()
    tol = 1e-13 if storage == "f64" else 1e-6
    print(f"  {storage}: |dM|/M = {abs(d['mass'] - m0) / m0:.3e}")
    assert abs(d["mass"] - m0) / m0 < tol
    assert d["status"] == 0 and d["nonfinite"] == 0


def test_fp64_200_step_prefix_laplace_128():
    """The 128^3 Laplace droplet in FP64, in its tuned launch configuration:
    every population after 200 steps against the oracle, to 1e-12."""
    import os
    _need_gpu()
    cfg, init = li.c2_laplace(20)
    cfg = dict(cfg, storage="f64")
    rho, u = li.init_fields(cfg, init)
    mode = tuning.mode_for("laplace_128", "f64")
    tile = tuning.tile_for("laplace_128", "f64", mode)
    got = gpu_states(cfg, rho, u, [200], tile, mode)[0]
    p = ref.make_params(cfg, nthreads=min(16, os.cpu_count() or 1))
    want = ref.step(p, ref.equilibrium(p, rho, u), 200)
    e = rho_err(got, want)
    print(f"  200 steps: err {e:.3e}", flush=True)
    assert e < 1e-12


@pytest.mark.parametrize("workload,storage", [("two_droplets_256", "f64"), ("two_droplets_256", "f32"),
                                              ("sessile_384x384x192", "f32")])
def test_full_size_mass_over_200_steps(workload, storage):
    """Mass is an exact invariant of the step (periodic, or half-way
    bounce-back walls): at full size in the tuned configuration, 200 steps
    move it by rounding only."""
    _need_gpu()
    cfg, init = FULL[workload]()
    cfg = dict(cfg, storage=storage)
    mode = tuning.mode_for(workload, storage)
    tile = tuning.tile_for(workload, storage, mode)
    print(f"[gpu] mass {workload} {storage} mode={mode} tile={tile}", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode(mode)
    if tile:
        lat.set_tile(*tile)
    lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"])
    m0 = lat.diagnostics()["mass"]
    lat.step(200)
    d = lat.diagnostics()
    lat.close()
    rel = abs(d["mass"] - m0) / m0
    print(f"  |dM|/M = {rel:.3e}")
    assert d["status"] == 0 and d["nonfinite"] == 0
    assert rel < (1e-13 if storage == "f64" else 1e-6)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_save_load_resume_is_bit_identical(storage):
    _need_gpu()
    cfg, init = li.c1_droplet()
    cfg = dict(cfg, storage=storage, rho_ref=init["rho_V"])
    a = Lattice(cfg)
    a.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"]).step(7)
    buf = a.save_state()
    a.step(7)
    fa = a.read_populations().cpu().numpy()
    b = Lattice(cfg)
    b.load_state(buf)
    assert b.steps == 7
    b.step(7)
    fb = b.read_populations().cpu().numpy()
    assert np.array_equal(fa, fb)
    a.close()
    b.close()


@pytest.mark.parametrize("storage,mode", [("f32", "pairs"), ("f32", "split"), ("f16s", "split"), ("f64", "fused")])
def test_autotune_leaves_state_unchanged(storage, mode):
    """The autotuner times candidate tiles of the current step mode by
    writing the other buffer only, and keeps a tile valid for that mode."""
    _need_gpu()
    cfg, init = li.c1_droplet()
    cfg = dict(cfg, storage=storage, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
    lat = Lattice(cfg)
    lat.set_step_mode(mode)
    lat.init_droplets(init["droplets"], init["rho_L"], init["rho_V"], init["W"]).step(2)
    f0 = lat.read_populations().cpu().numpy()
    t = lat.autotune(trials=1)
    assert lat.get_tile() == t
    lat.set_tile(*t)  # valid for the mode
    f1 = lat.read_populations().cpu().numpy()
    assert np.array_equal(f0, f1)
    lat.step(1)
    lat.close()


def test_nonfinite_detected():
    _need_gpu()
    cfg, init = li.c1_droplet(n=16, r0=4.0)
    cfg = dict(cfg, nx=16, ny=16, nz=16, storage="f32")
    lat = Lattice(cfg)
    rho, u = li.init_fields(cfg, init)
    f = ref.equilibrium(ref.make_params(cfg), rho, u)
    f[3, 100] = np.nan
    lat.write_populations(f)
    d = lat.diagnostics()
    assert d["status"] == -4 and d["nonfinite"] >= 1
    lat.close()


# ---------------------------------------------------------------------------
# Full-size workloads in their benchmark launch shape: one step from the
# initial condition, compared at sampled nodes computed one by one.
# ---------------------------------------------------------------------------
FULL = {
    "laplace_128": lambda: li.c2_laplace(20),
    "two_droplets_256": lambda: li.c3_two_droplets(),
    "sessile_384x384x192": lambda: li.c4_sessile(60.0),
}


@pytest.mark.parametrize("workload,storage", [("laplace_128", "f64"), ("laplace_128", "f32"),
                                              ("two_droplets_256", "f32"), ("sessile_384x384x192", "f32")])
def test_full_size_sampled_parity(workload, storage):
    """One step at sampled nodes (F16S: tests/test_gpu_f16s.py)."""
    _need_gpu()
    cfg, init = FULL[workload]()
    cfg = dict(cfg, storage=storage, rho_ref=init["rho_V"], f16_exp=f16_exp_for(1.25 * init["rho_L"]))
    rho, u = li.init_fields(cfg, init)
    N = rho.size
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([rng.integers(0, N, 3000),
                                    np.flatnonzero(np.abs(rho - 0.5 * (init["rho_L"] + init["rho_V"]))
                                                   < 0.25 * (init["rho_L"] - init["rho_V"]))[::97][:2000],
                                    [0, N - 1]]))
    mode = tuning.mode_for(workload, storage)
    tile = tuning.tile_for(workload, storage, mode)
    print(f"[gpu] {workload} {storage} mode={mode} tile={tile} samples={idx.size}", flush=True)
    lat = Lattice(cfg)
    lat.set_step_mode(mode)
    if tile:
        lat.set_tile(*tile)
    lat.init_fields(rho, u).step(1)
    f = lat.read_populations()
    got = f[:, torch.as_tensor(idx, device=f.device)].cpu().numpy().T
    lat.close()
    del f
    p = ref.make_params(cfg)
    f0 = ref.equilibrium(p, rho, u)
    want = ref.step_sampled(p, f0, idx)
    r = want.sum(1)
    err = np.abs(got - want)
    bound = (1e-12 if storage == "f64" else fp32_bound(1)) * r[:, None]
    print(f"  max err/rho {float((err / r[:, None]).max()):.3e}")
    assert np.all(err <= bound)


# ---------------------------------------------------------------------------
# Single-phase runs with walls on x and y and a moving lid (Appendix B cavity)
# ---------------------------------------------------------------------------
def _cavity(nx, ny, nz, op, storage, walls=(1, 1, 1), lid=(0.05, 0.0, 0.0), seed=21):
    cfg = li.params(nx, ny, nz, op=op, storage=storage, psi_form="exp", G=0.0, sigma=0.0, s_e=1.1,
                    tau_nu=0.8, wall_x=walls[0], wall_y=walls[1], wall_z=walls[2], lid_u=lid, lid_rho=1.0,
                    gravity=(0.0, 0.0, 1e-5))
    rho, u = li.random_fields(nx, ny, nz, seed=seed, rho_lo=0.95, rho_hi=1.05, umax=0.02)
    return cfg, rho, u


@pytest.mark.parametrize("op", ["nonorth", "orth"])
@pytest.mark.parametrize("walls", [(1, 1, 1), (1, 0, 0), (0, 1, 0), (1, 1, 0)])
def test_cavity_fp64_parity(op, walls):
    cfg, rho, u = _cavity(12, 10, 9, op, "f64", walls, lid=(0.05, 0.0, 0.0) if walls[1] else (0.0, 0.0, 0.0))
    cps = [0, 1, 5]
    got = gpu_states(cfg, rho, u, cps)
    want = oracle_states(cfg, rho, u, cps)
    for s, g, w in zip(cps, got, want):
        e = rho_err(g, w)
        print(f"  step {s}: err {e:.3e}")
        assert e < 1e-12, (s, e)


def test_cavity_fp32_parity():
    """The cavity in FP32 (F16S: tests/test_gpu_f16s.py)."""
    cfg, rho, u = _cavity(16, 12, 10, "nonorth", "f32")
    cps = [1, 10]
    got = gpu_states(cfg, rho, u, cps)
    want = oracle_states(cfg, rho, u, cps)
    for s, g, w in zip(cps, got, want):
        e = rho_err(g, w)
        print(f"  step {s}: err {e:.3e} (bound {fp32_bound(s):.1e})")
        assert e < fp32_bound(s), (s, e)


def test_cavity_write_read_round_trip_and_mass():
    _need_gpu()
    cfg, rho, u = _cavity(11, 9, 7, "nonorth", "f64")
    p = ref.make_params(cfg)
    f0 = ref.equilibrium(p, rho, u)
    lat = Lattice(cfg)
    lat.write_populations(f0)
    back = lat.read_populations().cpu().numpy()
    # populations reflected off the lid are stored as v - t and read as (v - t) + t
    assert np.abs(back - f0).max() < 1e-15
    cfg0 = dict(cfg, gravity=(0.0, 0.0, 0.0))
    lat.close()
    lat = Lattice(cfg0)
    lat.write_populations(f0)
    m0 = lat.diagnostics()["mass"]
    lat.step(300)
    m1 = lat.diagnostics()["mass"]
    lat.close()
    assert abs(m1 - m0) < 1e-12 * m0


def test_cavity_rejections():
    _need_gpu()
    with pytest.raises(binding.LbmError) as e:
        Lattice(li.params(16, 16, 16, wall_x=1))  # multiphase with x walls
    assert e.value.status == -5
    with pytest.raises(binding.LbmError) as e:
        Lattice(li.params(16, 16, 16, psi_form="exp", G=0.0, lid_u=(0.1, 0.0, 0.0)))  # lid without wall_y
    assert e.value.status == -1
    cfg, _, _ = _cavity(8, 8, 8, "nonorth", "f32")
    lat = Lattice(cfg)
    assert lat.step_mode() == "fused"
    with pytest.raises(binding.LbmError) as e:
        lat.set_step_mode("pairs")
    assert e.value.status == -5
    lat.close()
    with pytest.raises(binding.LbmError) as e:
        binding.Batch([cfg])
    assert e.value.status == -5


def test_diagnostics_are_deterministic():
    """The two-pass FP64 reduction has a fixed order: repeated calls on the
    same state give the same bits."""
    cfg, rho, u, tile = _case("ragged_70x37x21", "nonorth", "f32")
    _need_gpu()
    lat = Lattice(cfg)
    lat.init_fields(rho, u).step(3)
    c = (35.0, 18.5, 10.0)
    d1 = lat.diagnostics(center=c, r_in=5.0, r_out=15.0)
    d2 = lat.diagnostics(center=c, r_in=5.0, r_out=15.0)
    lat.close()
    for k in ("mass", "momentum", "max_u", "p_in", "p_out", "rho_in", "rho_out", "n_in", "n_out"):
        assert d1[k] == d2[k], k


# ---------------------------------------------------------------------------
# Write check: the destination buffer is filled with NaN before every step,
# so any node a step kernel leaves unwritten would surface as non-finite and
# break bit identity with the unchecked run.
# ---------------------------------------------------------------------------
WRITE_CHECK_CASES = [("ragged_70x37x21", "f32", "fused", None), ("ragged_70x37x21", "f16s", "pairs", (32, 4, 7)),
                     ("walls_40x33x19_60deg", "f64", "fused", None),
                     ("walls_40x33x19_60deg", "f32", "pairs", (16, 8, 7)),
                     ("walls_37x20x12_120deg", "f32", "slabs", None), ("cavity", "f32", "fused", None),
                     ("ragged_68x37x21", "f16s", "quads", (32, 4, 7)),
                     ("walls_40x33x19_60deg", "f16s", "quads", (40, 4, 7)),
                     ("ragged_68x37x21", "f16s", "split", (32, 4, 7)),
                     ("walls_40x33x19_60deg", "f16s", "split", (40, 4, 7)),
                     ("ragged_70x37x21", "f32", "split", (32, 4, 7))]


@pytest.mark.parametrize("name,storage,mode,tile", WRITE_CHECK_CASES)
def test_every_node_written_each_step(name, storage, mode, tile):
    _need_gpu()
    if name == "cavity":
        cfg, rho, u = _cavity(14, 11, 9, "nonorth", storage)
    else:
        cfg, rho, u, ctile = _case(name, "nonorth", storage)
        tile = tile or ctile
    print(f"[gpu] write check {name} {storage} {mode} tile={tile}", flush=True)
    out = []
    for check in (False, True):
        lat = Lattice(cfg)
        if mode == "slabs":
            lat.set_step_mode("slabs", 5)
        elif mode in ("pairs", "quads", "split"):
            lat.set_step_mode(mode)
        if tile is not None:
            lat.set_tile(*tile)
        lat.set_write_check(check)
        lat.init_fields(rho, u).step(3)
        d = lat.diagnostics()
        assert d["status"] == 0 and d["nonfinite"] == 0
        out.append(lat.read_populations().cpu().numpy())
        lat.close()
    assert np.isfinite(out[1]).all()
    assert np.array_equal(out[0], out[1])


def test_divergence_detected_on_device():
    """The unstable low-viscosity droplet (T = 0.5 T_c, s_nu = 1.9) is flagged
    non-finite by the device diagnostics; the stable one (s_nu = 1) stays
    finite over 1000 steps and ends with the oracle's maximum velocity."""
    _need_gpu()
    cfg, init = li.cold_droplet(1.9)
    print("[gpu] divergence s_nu=1.9 16^3 f64", flush=True)
    lat = Lattice(cfg)
    lat.init_fields(*li.init_fields(cfg, init)).step(100)
    d = lat.diagnostics()
    lat.close()
    assert d["status"] == -4 and d["nonfinite"] > 0
    cfg, init = li.cold_droplet(1.0)
    rho, u = li.init_fields(cfg, init)
    lat = Lattice(cfg)
    lat.init_fields(rho, u).step(1000)
    d = lat.diagnostics()
    lat.close()
    p = ref.make_params(cfg)
    fl = ref.fields(p, ref.step(p, ref.equilibrium(p, rho, u), 1000))
    want = float(np.sqrt((fl["u"] ** 2).sum(0)).max())
    assert d["status"] == 0 and abs(d["max_u"] - want) <= 1e-8 * want


# ---------------------------------------------------------------------------
# Degenerate shapes: lattices one or two nodes thick along some axes.  With
# n = 1 every stencil and streaming offset along that axis wraps onto the node
# itself; with n = 2 both neighbours are the same node.  Walls need two planes.
# ---------------------------------------------------------------------------
DEGENERATE = [(1, 1, 24, 0), (24, 1, 1, 0), (1, 17, 1, 0), (6, 4, 1, 0), (5, 1, 9, 1), (2, 3, 2, 1),
              (1, 1, 2, 1)]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny,nz,wall", DEGENERATE)
def test_degenerate_shapes_parity(nx, ny, nz, wall, storage):
    cfg = li.params(nx, ny, nz, T_over_Tc=0.8, storage=storage, wall_z=wall,
                    theta_wall_deg=70.0 if wall else 90.0)
    rho, u = li.random_fields(nx, ny, nz, seed=100 * nx + 10 * ny + nz, rho_lo=0.05, rho_hi=0.3, umax=0.03)
    cps = [1, 4]
    got = gpu_states(cfg, rho, u, cps)
    want = oracle_states(cfg, rho, u, cps)
    for s, g, w in zip(cps, got, want):
        e = rho_err(g, w)
        bound = 1e-12 if storage == "f64" else fp32_bound(s)
        print(f"  step {s}: err {e:.3e} (bound {bound:.1e})")
        assert e < bound, (s, e)


def test_zero_steps_change_nothing():
    """Stepping by zero is a no-op for a lattice and for a batch."""
    _need_gpu()
    cfg, rho, u, _ = _case("droplet_32", "nonorth", "f32")
    lat = Lattice(cfg)
    lat.init_fields(rho, u).step(2)
    f0 = lat.read_populations().cpu().numpy()
    n0 = lat.diagnostics()["step"]
    lat.step(0)
    assert lat.diagnostics()["step"] == n0 == 2
    assert np.array_equal(lat.read_populations().cpu().numpy(), f0)
    lat.close()
    b = binding.Batch([cfg, cfg])
    b.init_fields(0, rho, u)
    b.init_fields(1, rho, u)
    b.step(1, 0)
    g0 = b.read_populations(1).cpu().numpy()
    b.step(0, 4)
    assert np.array_equal(b.read_populations(1).cpu().numpy(), g0)
    assert b.diagnostics(1)["step"] == 1
    b.close()


# ---------------------------------------------------------------------------
# Largest lattices the 32-bit buffer offsets allow (five direction planes
# under 4 GiB), one per storage format.  The initial fields repeat with period
# 64 x 64 x P, so the large lattice must reproduce, bit for bit, the small
# periodic lattice at every sampled node; the small one is pinned to the
# oracle.
# ---------------------------------------------------------------------------
MAX_SHAPES = {"f64": ((640, 640, 262), 2), "f32": ((640, 640, 524), 4), "f16s": ((640, 640, 1048), 4)}


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_maximum_size_lattice(storage):
    _need_gpu()
    (nx, ny, nz), P = MAX_SHAPES[storage]
    E = {"f64": 8, "f32": 4, "f16s": 2}[storage]
    assert 5 * nx * ny * nz * E < 2 ** 32 <= 5 * nx * ny * (nz + 1) * E
    small = li.params(64, 64, P, T_over_Tc=0.8, storage=storage)
    if storage == "f16s":
        small.update(rho_ref=li.coexistence(0.8)[1], f16_exp=f16_exp_for(1.25 * 0.3))
    big = dict(small, nx=nx, ny=ny, nz=nz)
    rho, u = li.random_fields(64, 64, P, seed=77, rho_lo=0.05, rho_hi=0.3, umax=0.03)
    steps = 2
    fs = gpu_states(small, rho, u, [steps])[0]
    if storage == "f64":
        want = oracle_states(small, rho, u, [steps])[0]
        assert rho_err(fs, want) < 1e-12
    reps = (nz // P, ny // 64, nx // 64)
    rho_b = np.tile(rho.reshape(P, 64, 64), reps).reshape(-1)
    u_b = np.tile(u.reshape(3, P, 64, 64), (1,) + reps).reshape(3, -1)
    N = nx * ny * nz
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.integers(0, N, 4000), [0, nx - 1, nx * ny - 1, N - nx * ny, N - 1]]))
    print(f"[gpu] max size {nx}x{ny}x{nz} {storage} samples={idx.size}", flush=True)
    lat = Lattice(big)
    assert lat.N == N
    lat.init_fields(rho_b, u_b)
    del rho_b, u_b
    lat.step(steps)
    f = lat.read_populations()
    got = f[:, torch.as_tensor(idx, device=f.device)].cpu().numpy()
    del f
    lat.close()
    torch.cuda.empty_cache()
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    src = ((z % P) * 64 + y % 64) * 64 + x % 64
    assert np.array_equal(got, fs[:, src])


# ---------------------------------------------------------------------------
# Readings of the orthogonal comparison operator: the alternative equilibrium
# of its eps and pi rows (orth_meq = 1) and the Eq. (16) term on the e row
# only (orth_sigma = 1), against the oracle with the same reading.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("meq,sig", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("name", ["droplet_32", "walls_40x33x19_60deg"])
def test_orth_readings_parity(name, meq, sig):
    cfg, rho, u, tile = _case(name, "orth", "f64")
    cfg = dict(cfg, orth_meq=meq, orth_sigma=sig)
    cps = [0, 1, 5, 50]
    got = gpu_states(cfg, rho, u, cps, tile)
    want = oracle_states(cfg, rho, u, cps)
    for s, g, w in zip(cps, got, want):
        e = rho_err(g, w)
        print(f"  step {s}: err {e:.3e}")
        assert e < 1e-12, (s, e)
    cfg32 = dict(cfg, storage="f32")
    got = gpu_states(cfg32, rho, u, [1, 10], None, "split")
    want = oracle_states(cfg32, rho, u, [1, 10])
    for s, g, w in zip([1, 10], got, want):
        assert rho_err(g, w) < fp32_bound(s), s
