"""Host sanitizers (AddressSanitizer, UndefinedBehaviorSanitizer) over the C
oracle and over the host side of the HIP library's C ABI, built on the CPU.

* The oracle, linked into tests/sanitize/oracle_driver.c with -fsanitize,
  steps periodic, walled, orthogonal, exponential-psi, variable-viscosity and
  lid-driven-cavity lattices (including one- and two-node-thick axes); the
  results must also equal the regular oracle build bit for bit.
* The library's host code (parameter validation, workspace layout, context
  and batch set-up, launch-shape and mode checks, the argument checks of
  every entry point) runs in tests/sanitize/runtime_driver.cpp with host
  sanitizers; device code is compiled without any sanitizer and never runs.
Any sanitizer report aborts the program (halt_on_error), so a zero exit
status means a clean run.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import lbm_inputs as li
from oracle import build as obuild
from oracle import ref

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


@pytest.fixture(scope="module")
def oracle_driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("asan_oracle")
    exe = os.path.join(d, "oracle_driver")
    cmd = ["gcc", *[f for f in obuild.CFLAGS if f != "-O2"], "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           obuild.SRC, os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True)
    return exe


CASES = {
    "periodic_nonorth": lambda: li.params(9, 7, 6, T_over_Tc=0.8, sigma=0.105),
    "periodic_orth": lambda: li.params(9, 7, 6, T_over_Tc=0.8, sigma=0.105, op="orth"),
    "walls_gravity_60deg": lambda: li.params(8, 6, 7, T_over_Tc=0.7, wall_z=1, theta_wall_deg=60.0,
                                            gravity=(0.0, 0.0, -1e-5), ghost_rho_min=0.01),
    "exp_psi_walls_120deg": lambda: li.params(8, 6, 5, psi_form="exp", G=-10.0 / 3.0, psi0=1.0, rho0=1.0,
                                             wall_z=1, theta_wall_deg=120.0, sigma=0.0),
    "variable_viscosity": lambda: li.params(7, 6, 5, T_over_Tc=0.6, eos_a=0.25, tau_nu=0.53, nu_ratio=10.0,
                                           visc_rho_L=0.4, visc_rho_V=0.003),
    "cavity_lid": lambda: li.params(6, 5, 4, psi_form="exp", G=0.0, sigma=0.0, wall_x=1, wall_y=1, wall_z=1,
                                   lid_u=(0.05, 0.0, 0.0), lid_rho=1.0),
    "thin_axes": lambda: li.params(1, 2, 5, T_over_Tc=0.8, wall_z=1, theta_wall_deg=70.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_clean_under_sanitizers(oracle_driver, tmp_path, name):
    cfg = CASES[name]()
    p = ref.make_params(cfg)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    N = nx * ny * nz
    if cfg.get("psi_form") == "exp" and cfg["G"] == 0.0:
        rho, u = li.random_fields(nx, ny, nz, seed=5, rho_lo=0.95, rho_hi=1.05, umax=0.02)
    elif cfg.get("psi_form") == "exp":
        rho, u = li.random_fields(nx, ny, nz, seed=5, rho_lo=0.4, rho_hi=2.7, umax=0.02)
    else:
        rho, u = li.random_fields(nx, ny, nz, seed=5, rho_lo=0.05, rho_hi=0.3, umax=0.03)
    f = ref.equilibrium(p, rho, u)
    pf, ff, of = (os.path.join(tmp_path, n) for n in ("params.bin", "f.bin", "out.bin"))
    with open(pf, "wb") as fh:
        fh.write(ctypes.string_at(ctypes.byref(p), ctypes.sizeof(p)))
    f.astype(np.float64).tofile(ff)
    r = subprocess.run([oracle_driver, pf, ff, of, "3"], env=ENV, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    out = np.fromfile(of, dtype=np.float64)
    ns = min(N, 64)
    step = out[:19 * N].reshape(19, N)
    fields = out[19 * N:28 * N]
    coll = out[28 * N:28 * N + 19 * ns].reshape(ns, 19)
    eq = out[28 * N + 19 * ns:].reshape(19, N)
    # Same arithmetic as the regular build, bit for bit.
    assert np.array_equal(step, ref.step(p, f, 3))
    fl = ref.fields(p, f)
    assert np.array_equal(fields[:N], fl["rho"]) and np.array_equal(fields[4 * N:7 * N], fl["F"].reshape(-1))
    assert np.array_equal(coll, ref.collide_nodes(p, f, np.arange(ns)))
    assert np.array_equal(eq, ref.equilibrium(p, fl["rho"], np.zeros((3, N))))


def test_runtime_host_paths_clean_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = os.path.join(tmp_path, "runtime_driver")
    # Host code with the sanitizers, device code without (and at -O0: it is
    # compiled only to link, and never runs here).
    cmd = [hipcc, "--offload-arch=gfx950", "-std=c++17", "-g", "-Xarch_host", "-O1", "-Xarch_device", "-O0",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "paper_1805_08643_amd", "csrc", "lbm_api.hip"),
           os.path.join(HERE, "sanitize", "runtime_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True)
    print(r.stdout[-2000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "OK: 0 failure(s)" in r.stdout
