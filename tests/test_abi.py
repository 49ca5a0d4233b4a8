"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1805_08643_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(header="mrt_lbm.h"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = header_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert sorted(binding.SIGNATURES) == names


def test_probe_library_exports_every_declared_symbol():
    from paper_1805_08643_amd import probe
    L = probe.lib()
    names = header_functions("mrt_probe.h")
    assert names == sorted(probe.SIGNATURES)
    for n in names:
        assert hasattr(L, n), n


def test_every_header_is_covered():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["mrt_lbm.h", "mrt_probe.h"]


def test_probe_rejects_bad_arguments_before_any_launch():
    from paper_1805_08643_amd import probe
    with pytest.raises(binding.LbmError):
        probe.lbm_probe_copy(256, 256, 1024, 0, 0, 0)  # same buffer
    with pytest.raises(binding.LbmError):
        probe.lbm_probe_copy(256, 512, 1000, 0, 0, 0)  # not a multiple of 16
    with pytest.raises(binding.LbmError):
        probe.lbm_probe_stream19(256, 512, 1024, 12, 0, 0, 0)  # group size
    with pytest.raises(binding.LbmError):
        probe.lbm_probe_march19(256, 512, 8, 8, 8, 8, 64, 32, 8, 0, 0)  # tx * ty > 1024
    with pytest.raises(binding.LbmError):
        probe.lbm_probe_march19(264, 512, 8, 8, 8, 8, 8, 8, 8, 0, 0)  # misaligned


def test_params_default_and_workspace_size():
    p = binding.lbm_params_default()
    assert (p.nx, p.ny, p.nz) == (32, 32, 32) and p.G == -1.0 and p.eos_b == 4.0
    n = binding.lbm_workspace_bytes(p)
    N = 32 ** 3
    pops = 19 * N * 4
    assert n >= 2 * pops + N * 4
    p.storage = binding.STORAGE["f16s"]
    assert binding.lbm_workspace_bytes(p) < n
    p.storage = binding.STORAGE["f64"]
    assert binding.lbm_workspace_bytes(p) > n


@pytest.mark.parametrize("field,value", [("nx", 0), ("s_nu", 2.0), ("s_e", 0.0), ("G", 0.5), ("op", 7),
                                         ("storage", 9), ("T_over_Tc", -1.0), ("theta_wall_deg", 180.0),
                                         ("f16_exp", 30), ("nu_ratio", -1.0), ("nu_ratio", float("nan"))])
def test_invalid_params_rejected(field, value):
    p = binding.lbm_params_default()
    setattr(p, field, value)
    n = ctypes.c_size_t(0)
    st = binding.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    assert st == -1
    assert binding.lbm_last_error()


def test_variable_viscosity_needs_density_range():
    p = binding.lbm_params_default()
    n = ctypes.c_size_t(0)
    p.nu_ratio = 10.0
    p.visc_rho_L, p.visc_rho_V = 0.1, 0.4  # inverted
    assert binding.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == -1
    p.visc_rho_L, p.visc_rho_V = 0.4, 0.003
    assert binding.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    p.nu_ratio, p.visc_rho_L, p.visc_rho_V = 1.0, 0.0, 0.0  # uniform: range unused
    assert binding.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == 0


def test_walls_need_two_planes():
    p = binding.lbm_params_default()
    p.wall_z, p.nz = 1, 1
    n = ctypes.c_size_t(0)
    assert binding.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == -1


def test_create_rejects_small_or_misaligned_workspace_without_gpu():
    p = binding.lbm_params_default()
    need = binding.lbm_workspace_bytes(p)
    ctx = ctypes.c_void_p()
    L = binding.lib()
    st = L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4096), need - 1, None, ctypes.byref(ctx))
    assert st == -2 and not ctx.value
    st = L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4096 + 8), need, None, ctypes.byref(ctx))
    assert st == -1
    st = L.lbm_create(ctypes.byref(p), None, need, None, ctypes.byref(ctx))
    assert st == -1


def test_batch_validation():
    a = binding.lbm_params_default()
    b = binding.lbm_params_default()
    b.op = binding.OP["orth"]
    arr = (binding.LbmParams * 2)(a, b)
    n = ctypes.c_size_t(0)
    assert binding.lib().lbm_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == -1
    b.op = a.op
    b.wall_z = 1
    arr = (binding.LbmParams * 2)(a, b)
    assert binding.lib().lbm_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == -5
    arr = (binding.LbmParams * 2)(a, a)
    assert binding.lib().lbm_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == 0
    assert n.value >= 2 * binding.lbm_workspace_bytes(a)


def test_batch_tuning_calls_reject_null():
    L = binding.lib()
    m = ctypes.c_int32(0)
    assert L.lbm_batch_set_item_nodes(None, 4096) == -1
    assert L.lbm_batch_get_tuning(None, ctypes.byref(m), None, None) == -1


def test_status_strings():
    assert binding.lbm_status_string(0) == "ok"
    assert binding.lbm_status_string(-4) == "non-finite populations"


def test_make_params_mapping():
    p = binding.make_params(dict(nx=8, ny=9, nz=10, tau_nu=0.8, s_e=1.1, s_q=1.2, s_pi=1.4, op="orth",
                                 storage="f16s", rho_ref=0.01, gravity=(0, 0, -1e-6), wall_z=1))
    assert (p.nx, p.ny, p.nz, p.wall_z, p.op, p.storage) == (8, 9, 10, 1, 1, 2)
    assert p.s_nu == 1.25 and p.s_eps == 1.4 and p.s_m == 1.2 and p.gravity[2] == -1e-6


def test_f16n_layout_and_limits():
    """F16N holds a twentieth plane (the reference densities) beside the 19
    populations of 2 bytes, and the seed of its stochastic rounding after
    them, and runs the split step only: nx a multiple of 4, walls only on z
    (batches of such runs too)."""
    p = binding.lbm_params_default()
    p.storage = binding.STORAGE["f16s"]
    n16s = binding.lbm_workspace_bytes(p)
    p.storage = binding.STORAGE["f16n"]
    n16n = binding.lbm_workspace_bytes(p)
    # one more plane of 2-byte values and the 16-byte rounding seed in each of the two buffers (256-byte aligned)
    assert n16n - n16s == 2 * ((20 * 32 ** 3 * 2 + 16 + 255) // 256 * 256 - 19 * 32 ** 3 * 2)
    assert binding.population_bytes("f16n", 32 ** 3) == 20 * 32 ** 3 * 2 + 16
    n = ctypes.c_size_t(0)
    L = binding.lib()
    p.nx = 30
    assert L.lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == -5
    assert "F16N" in binding.lbm_last_error()
    p.nx = 32
    p.wall_z = 1
    assert L.lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    p.wall_z, p.wall_x = 0, 1
    assert L.lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == -5
    p.wall_x = 0
    arr = (binding.LbmParams * 2)(p, p)
    assert L.lbm_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == 0
    assert n.value >= 2 * n16n
    assert binding.algorithmic_bytes_per_node("f16n") == 80


@pytest.mark.parametrize("storage,nz_max", [("f64", 262), ("f32", 524), ("f16s", 1048), ("f16n", 1048)])
def test_largest_lattice_accepted_next_rejected(storage, nz_max):
    """Five direction planes must fit the 32-bit buffer offsets (< 4 GiB):
    640 x 640 x nz_max is the largest such lattice, one plane more is not."""
    p = binding.lbm_params_default()
    p.nx, p.ny, p.nz = 640, 640, nz_max
    p.storage = binding.STORAGE[storage]
    n = ctypes.c_size_t(0)
    assert binding.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    p.nz = nz_max + 1
    assert binding.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == -5
    assert "too large" in binding.lbm_last_error()


def test_source_digest_counts_code_not_comments():
    """The digest that ties stored profiles to the kernel sources sees their
    code only: comments and layout do not change it, code does, and literals
    that look like comments are code."""
    from paper_1805_08643_amd.build import code_text
    a = "int f(int x) {\n  return x + 1; // one more\n}\n"
    b = "/* the same */ int f(int x)   { return x + 1; }"
    c = "int f(int x) { return x + 2; }"
    assert code_text(a) == code_text(b) != code_text(c)
    assert code_text('const char *s = "a // b /* c";') == 'const char *s = "a // b /* c";'
    assert code_text("char q = '\\'';  // quote") == "char q = '\\'';"
