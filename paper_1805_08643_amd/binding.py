"""Thin ctypes binding of ``include/mrt_lbm.h``.

Functions keep the C names (``lbm_create``, ``lbm_step``, ...) and only
marshal arguments: device buffers are torch tensors on the GPU (passed by
``data_ptr()``), the stream is torch's current stream.  Every step of the
lattice update runs in the HIP library; if ``lib/libmrtlbm.so`` is missing
this module raises instead of falling back to anything else.

``Lattice`` and ``Batch`` wrap a context with the workspace tensor that
backs it.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libmrtlbm.so")

Q = 19
OP = {"nonorth": 0, "orth": 1}
STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "f16n": 3}
PSI = {"sqrt_cs": 0, "exp": 1}
STEP_MODES = {"fused": 0, "slabs": 1, "pairs": 2, "quads": 3, "split": 4}
STORE_POLICIES = {"auto": 0, "cached": 1, "stream": 2}


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("wall_z", ctypes.c_int32), ("op", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("psi_form", ctypes.c_int32), ("f16_exp", ctypes.c_int32),
        ("rho_ref", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_nu", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_pi", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_m", ctypes.c_double),
        ("G", ctypes.c_double), ("eos_a", ctypes.c_double), ("eos_b", ctypes.c_double),
        ("eos_R", ctypes.c_double), ("T_over_Tc", ctypes.c_double),
        ("psi0", ctypes.c_double), ("rho0", ctypes.c_double), ("sigma", ctypes.c_double),
        ("gravity", ctypes.c_double * 3), ("theta_wall_deg", ctypes.c_double),
        ("ghost_rho_min", ctypes.c_double),
        ("nu_ratio", ctypes.c_double), ("visc_rho_L", ctypes.c_double), ("visc_rho_V", ctypes.c_double),
        ("wall_x", ctypes.c_int32), ("wall_y", ctypes.c_int32),
        ("lid_u", ctypes.c_double * 3), ("lid_rho", ctypes.c_double),
        ("diag_every", ctypes.c_int32), ("orth_meq", ctypes.c_int32), ("orth_sigma", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
    ]


class LbmTile(ctypes.Structure):
    _fields_ = [("tx", ctypes.c_int32), ("ty", ctypes.c_int32), ("cz", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class LbmDroplet(ctypes.Structure):
    _fields_ = [("center", ctypes.c_double * 3), ("r0", ctypes.c_double), ("u", ctypes.c_double * 3)]


class LbmDiagRequest(ctypes.Structure):
    _fields_ = [("center", ctypes.c_double * 3), ("r_in", ctypes.c_double), ("r_out", ctypes.c_double)]


class LbmDiag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3), ("max_u", ctypes.c_double),
                ("p_in", ctypes.c_double), ("p_out", ctypes.c_double), ("rho_in", ctypes.c_double),
                ("rho_out", ctypes.c_double), ("n_in", ctypes.c_double), ("n_out", ctypes.c_double),
                ("nonfinite", ctypes.c_int64), ("step", ctypes.c_int64)]


class LbmError(RuntimeError):
    def __init__(self, status, fn, msg):
        super().__init__(f"{fn}: status {status}: {msg}")
        self.status = status


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_dp = _P(ctypes.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "lbm_params_default": (None, [_P(LbmParams)]),
    "lbm_workspace_bytes": (_i32, [_P(LbmParams), _P(_sz)]),
    "lbm_create": (_i32, [_P(LbmParams), _vp, _sz, _vp, _P(_vp)]),
    "lbm_destroy": (_i32, [_vp]),
    "lbm_init_fields": (_i32, [_vp, _vp, _vp]),
    "lbm_init_droplets": (_i32, [_vp, _P(LbmDroplet), _i32, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lbm_step": (_i32, [_vp, _i64]),
    "lbm_read_fields": (_i32, [_vp, _vp, _vp, _vp]),
    "lbm_read_populations": (_i32, [_vp, _vp]),
    "lbm_write_populations": (_i32, [_vp, _vp]),
    "lbm_diagnostics": (_i32, [_vp, _P(LbmDiagRequest), _P(LbmDiag)]),
    "lbm_state_bytes": (_i32, [_vp, _P(_sz)]),
    "lbm_save_state": (_i32, [_vp, _vp, _sz]),
    "lbm_load_state": (_i32, [_vp, _vp, _sz]),
    "lbm_set_tile": (_i32, [_vp, _P(LbmTile)]),
    "lbm_get_tile": (_i32, [_vp, _P(LbmTile)]),
    "lbm_autotune": (_i32, [_vp, _i32, _P(LbmTile)]),
    "lbm_set_step_mode": (_i32, [_vp, _i32, _i32]),
    "lbm_get_step_mode": (_i32, [_vp, _P(_i32), _P(_i32)]),
    "lbm_set_timing": (_i32, [_vp, _i32]),
    "lbm_kernel_time": (_i32, [_vp, _dp, _P(_i64)]),
    "lbm_step_count": (_i64, [_vp]),
    "lbm_status_string": (ctypes.c_char_p, [_i32]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_batch_workspace_bytes": (_i32, [_P(LbmParams), _i32, _P(_sz)]),
    "lbm_batch_create": (_i32, [_P(LbmParams), _i32, _vp, _sz, _vp, _P(_vp)]),
    "lbm_batch_destroy": (_i32, [_vp]),
    "lbm_batch_init_droplets": (_i32, [_vp, _i32, _P(LbmDroplet), _i32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double]),
    "lbm_batch_init_fields": (_i32, [_vp, _i32, _vp, _vp]),
    "lbm_batch_step": (_i32, [_vp, _i64, _i32]),
    "lbm_batch_read_fields": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "lbm_batch_read_populations": (_i32, [_vp, _i32, _vp]),
    "lbm_batch_autotune": (_i32, [_vp, _i32, _P(_i32)]),
    "lbm_batch_set_blocks": (_i32, [_vp, _i32]),
    "lbm_batch_set_item_nodes": (_i32, [_vp, _i32]),
    "lbm_batch_get_tuning": (_i32, [_vp, _P(_i32), _P(_i32), _P(_i32)]),
    "lbm_batch_set_step_mode": (_i32, [_vp, _i32]),
    "lbm_batch_get_step_mode": (_i32, [_vp, _P(_i32)]),
    "lbm_batch_kernel_time": (_i32, [_vp, _dp, _P(_i64)]),
    "lbm_batch_nodes": (_i64, [_vp]),
    "lbm_set_write_check": (_i32, [_vp, _i32]),
    "lbm_set_store_policy": (_i32, [_vp, _i32]),
    "lbm_batch_set_store_policy": (_i32, [_vp, _i32]),
    "lbm_batch_diagnostics": (_i32, [_vp, _i32, _P(LbmDiagRequest), _P(LbmDiag)]),
    "lbm_batch_status": (_i32, [_vp, _P(_i32)]),
    "lbm_batch_runs": (_i32, [_vp]),
    "lbm_step_noalloc": (_i32, [_P(LbmParams), _vp, _vp, _vp]),
    "lbm_set_graph_steps": (_i32, [_vp, _i32]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} missing "
                               "(run __graft_entry__.build() or python paper_1805_08643_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, fn):
    if status != 0:
        msg = lib().lbm_last_error().decode(errors="replace")
        raise LbmError(status, fn, msg)


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    check(st, name)


# C-ABI names, argument marshalling only -------------------------------------
def lbm_params_default() -> LbmParams:
    p = LbmParams()
    lib().lbm_params_default(ctypes.byref(p))
    return p


def lbm_workspace_bytes(p: LbmParams) -> int:
    n = _sz(0)
    _call("lbm_workspace_bytes", ctypes.byref(p), ctypes.byref(n))
    return n.value


def lbm_create(p: LbmParams, ws_ptr: int, ws_bytes: int, stream: int) -> int:
    ctx = _vp()
    _call("lbm_create", ctypes.byref(p), _vp(ws_ptr), ws_bytes, _vp(stream), ctypes.byref(ctx))
    return ctx.value


def lbm_destroy(ctx):
    _call("lbm_destroy", _vp(ctx))


def lbm_init_fields(ctx, rho_ptr, u_ptr):
    _call("lbm_init_fields", _vp(ctx), _vp(rho_ptr), _vp(u_ptr))


def lbm_init_droplets(ctx, droplets, rho_L, rho_V, W):
    arr = _droplet_array(droplets)
    _call("lbm_init_droplets", _vp(ctx), arr, len(droplets), rho_L, rho_V, W)


def lbm_step(ctx, nsteps):
    _call("lbm_step", _vp(ctx), nsteps)


def lbm_step_noalloc(p: LbmParams, src_ptr: int, dst_ptr: int, stream: int):
    _call("lbm_step_noalloc", ctypes.byref(p), _vp(src_ptr), _vp(dst_ptr), _vp(stream))


def lbm_read_fields(ctx, rho_ptr, u_ptr, p_ptr):
    _call("lbm_read_fields", _vp(ctx), _vp(rho_ptr), _vp(u_ptr), _vp(p_ptr))


def lbm_read_populations(ctx, f_ptr):
    _call("lbm_read_populations", _vp(ctx), _vp(f_ptr))


def lbm_write_populations(ctx, f_ptr):
    _call("lbm_write_populations", _vp(ctx), _vp(f_ptr))


def lbm_diagnostics(ctx, req: LbmDiagRequest | None) -> tuple[int, LbmDiag]:
    d = LbmDiag()
    st = lib().lbm_diagnostics(_vp(ctx), ctypes.byref(req) if req is not None else None, ctypes.byref(d))
    if st not in (0, -4):
        check(st, "lbm_diagnostics")
    return st, d


def _diag_request(center, r_in, r_out):
    if center is None:
        return None
    req = LbmDiagRequest()
    for a in range(3):
        req.center[a] = float(center[a])
    req.r_in, req.r_out = float(r_in), float(r_out)
    return req


def _diag_dict(st, d):
    return {"status": st, "mass": d.mass, "momentum": tuple(d.momentum), "max_u": d.max_u,
            "p_in": d.p_in, "p_out": d.p_out, "rho_in": d.rho_in, "rho_out": d.rho_out,
            "n_in": d.n_in, "n_out": d.n_out, "nonfinite": d.nonfinite, "step": d.step}


def lbm_state_bytes(ctx) -> int:
    n = _sz(0)
    _call("lbm_state_bytes", _vp(ctx), ctypes.byref(n))
    return n.value


def lbm_save_state(ctx, ptr, nbytes):
    _call("lbm_save_state", _vp(ctx), _vp(ptr), nbytes)


def lbm_load_state(ctx, ptr, nbytes):
    _call("lbm_load_state", _vp(ctx), _vp(ptr), nbytes)


def lbm_set_tile(ctx, tx, ty, cz):
    t = LbmTile(tx, ty, cz, 0)
    _call("lbm_set_tile", _vp(ctx), ctypes.byref(t))


def lbm_get_tile(ctx):
    t = LbmTile()
    _call("lbm_get_tile", _vp(ctx), ctypes.byref(t))
    return (t.tx, t.ty, t.cz)


def lbm_autotune(ctx, trials):
    t = LbmTile()
    _call("lbm_autotune", _vp(ctx), trials, ctypes.byref(t))
    return (t.tx, t.ty, t.cz)


def lbm_set_step_mode(ctx, mode, slab_planes):
    _call("lbm_set_step_mode", _vp(ctx), int(mode), int(slab_planes))


def lbm_get_step_mode(ctx):
    m, sl = _i32(0), _i32(0)
    _call("lbm_get_step_mode", _vp(ctx), ctypes.byref(m), ctypes.byref(sl))
    return m.value, sl.value


def lbm_set_timing(ctx, enable):
    _call("lbm_set_timing", _vp(ctx), int(bool(enable)))


def lbm_kernel_time(ctx):
    ms = ctypes.c_double(0)
    n = _i64(0)
    _call("lbm_kernel_time", _vp(ctx), ctypes.byref(ms), ctypes.byref(n))
    return ms.value, n.value


def lbm_step_count(ctx) -> int:
    return lib().lbm_step_count(_vp(ctx))


def lbm_status_string(s) -> str:
    return lib().lbm_status_string(s).decode()


def lbm_last_error() -> str:
    return lib().lbm_last_error().decode(errors="replace")


# ----------------------------------------------------------------------------
def _droplet_array(droplets):
    arr = (LbmDroplet * len(droplets))()
    for k, d in enumerate(droplets):
        for a in range(3):
            arr[k].center[a] = float(d["center"][a])
            arr[k].u[a] = float(d.get("u", (0.0, 0.0, 0.0))[a])
        arr[k].r0 = float(d["r0"])
    return arr


def make_params(cfg: dict) -> LbmParams:
    """Workload dict (keys as in lbm_inputs) -> lbm_params."""
    p = lbm_params_default()
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
    p.wall_z = int(cfg.get("wall_z", 0))
    p.op = OP[cfg.get("op", "nonorth")]
    p.storage = STORAGE[cfg.get("storage", "f32")]
    p.psi_form = PSI[cfg.get("psi_form", "sqrt_cs")]
    p.rho_ref = float(cfg.get("rho_ref", 0.0))
    p.f16_exp = int(cfg.get("f16_exp", 0))
    s_nu = 1.0 / cfg["tau_nu"] if "tau_nu" in cfg else cfg.get("s_nu", 1.0)
    if "rates_all" in cfg:
        s = float(cfg["rates_all"])
        p.s_e = p.s_nu = p.s_q = p.s_pi = p.s_eps = p.s_m = s
    else:
        p.s_e = cfg.get("s_e", 1.0)
        p.s_nu = s_nu
        p.s_q = cfg.get("s_q", 1.0)
        p.s_pi = cfg.get("s_pi", 1.0)
        p.s_eps = cfg.get("s_eps", p.s_pi)
        p.s_m = cfg.get("s_m", p.s_q)
    p.G = cfg.get("G", -1.0)
    p.eos_a = cfg.get("eos_a", 0.5)
    p.eos_b = cfg.get("eos_b", 4.0)
    p.eos_R = cfg.get("eos_R", 1.0)
    p.T_over_Tc = cfg.get("T_over_Tc", 0.8)
    p.psi0 = cfg.get("psi0", 1.0)
    p.rho0 = cfg.get("rho0", 1.0)
    p.sigma = cfg.get("sigma", 0.0)
    g = cfg.get("gravity", (0.0, 0.0, 0.0))
    for d in range(3):
        p.gravity[d] = g[d]
    p.theta_wall_deg = cfg.get("theta_wall_deg", 90.0)
    p.ghost_rho_min = cfg.get("ghost_rho_min", 0.0)
    p.nu_ratio = cfg.get("nu_ratio", 0.0)
    p.visc_rho_L = cfg.get("visc_rho_L", 0.0)
    p.visc_rho_V = cfg.get("visc_rho_V", 0.0)
    p.wall_x = int(cfg.get("wall_x", 0))
    p.wall_y = int(cfg.get("wall_y", 0))
    lu = cfg.get("lid_u", (0.0, 0.0, 0.0))
    for d in range(3):
        p.lid_u[d] = lu[d]
    p.lid_rho = cfg.get("lid_rho", 1.0)
    p.diag_every = int(cfg.get("diag_every", 0))
    p.orth_meq = int(cfg.get("orth_meq", 0))
    p.orth_sigma = int(cfg.get("orth_sigma", 0))
    return p


def _torch():
    import torch
    return torch


class Lattice:
    """One lattice on a GPU, backed by a caller-owned workspace tensor."""

    def __init__(self, cfg: dict, device: str = "cuda:0"):
        torch = _torch()
        self.cfg = dict(cfg)
        self.params = make_params(cfg)
        self.device = torch.device(device)
        self.N = self.params.nx * self.params.ny * self.params.nz
        nbytes = lbm_workspace_bytes(self.params)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = lbm_create(self.params, self._ws_ptr, nbytes, self.stream.cuda_stream)

    # lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # helpers ------------------------------------------------------------------
    def _dev(self, a, shape):
        torch = _torch()
        t = torch.as_tensor(a, dtype=torch.float64).reshape(shape).to(self.device).contiguous()
        return t

    def init_fields(self, rho, u):
        r = self._dev(rho, (self.N,))
        v = self._dev(u, (3, self.N))
        lbm_init_fields(self.ctx, r.data_ptr(), v.data_ptr())
        self._keep = (r, v)
        return self

    def init_droplets(self, droplets, rho_L, rho_V, W):
        lbm_init_droplets(self.ctx, droplets, rho_L, rho_V, W)
        return self

    def step(self, n=1):
        lbm_step(self.ctx, int(n))
        return self

    def read_fields(self):
        torch = _torch()
        rho = torch.empty(self.N, dtype=torch.float64, device=self.device)
        u = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        p = torch.empty(self.N, dtype=torch.float64, device=self.device)
        lbm_read_fields(self.ctx, rho.data_ptr(), u.data_ptr(), p.data_ptr())
        return {"rho": rho, "u": u, "p": p}

    def read_populations(self):
        torch = _torch()
        f = torch.empty((Q, self.N), dtype=torch.float64, device=self.device)
        lbm_read_populations(self.ctx, f.data_ptr())
        return f

    def write_populations(self, f):
        t = self._dev(f, (Q, self.N))
        lbm_write_populations(self.ctx, t.data_ptr())
        self.stream.synchronize()
        return self

    def diagnostics(self, center=None, r_in=0.0, r_out=0.0):
        st, d = lbm_diagnostics(self.ctx, _diag_request(center, r_in, r_out))
        return _diag_dict(st, d)

    def save_state(self):
        torch = _torch()
        n = lbm_state_bytes(self.ctx)
        buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        lbm_save_state(self.ctx, buf.data_ptr(), n)
        return buf

    def load_state(self, buf):
        lbm_load_state(self.ctx, buf.data_ptr(), buf.numel())
        return self

    def set_tile(self, tx, ty, cz):
        lbm_set_tile(self.ctx, tx, ty, cz)

    def set_write_check(self, on=True):
        """Fill the destination buffer with NaN before every step (debug)."""
        _call("lbm_set_write_check", _vp(self.ctx), int(bool(on)))
        return self

    def set_store_policy(self, policy):
        """Split step's population stores: "auto", "cached" or "stream"."""
        _call("lbm_set_store_policy", _vp(self.ctx), STORE_POLICIES[policy])
        return self

    def get_tile(self):
        return lbm_get_tile(self.ctx)

    def autotune(self, trials=3):
        return lbm_autotune(self.ctx, trials)

    def set_step_mode(self, mode, slab_planes=32):
        """mode: "fused", "slabs", "pairs", "quads" or "split"."""
        lbm_set_step_mode(self.ctx, STEP_MODES[mode], slab_planes)
        return self

    def step_mode(self):
        m, _ = lbm_get_step_mode(self.ctx)
        return {v: k for k, v in STEP_MODES.items()}[m]

    def set_timing(self, on=True):
        lbm_set_timing(self.ctx, on)

    def set_graph_steps(self, k):
        """Replay runs of k steps from captured hipGraphs (0: plain launches)."""
        _call("lbm_set_graph_steps", _vp(self.ctx), int(k))
        return self

    def kernel_time(self):
        return lbm_kernel_time(self.ctx)

    @property
    def steps(self):
        return lbm_step_count(self.ctx)


def f16_exp_for(rho_max: float) -> int:
    """Exponent offset for shifted binary16 storage: the largest shifted
    population (at most the rest population rho_max / 3) scaled by 2^e stays
    below 2^15, so nothing overflows and small shifted values stay normal."""
    return int(math.floor(math.log2(2.0 ** 15 / (rho_max / 3.0))))


class Batch:
    """Many independent periodic lattices advanced by one persistent launch per
    step (common operator and storage), backed by one workspace tensor."""

    def __init__(self, cfgs, device: str = "cuda:0"):
        torch = _torch()
        self.cfgs = [dict(c) for c in cfgs]
        n = len(cfgs)
        self.params = (LbmParams * n)(*[make_params(c) for c in cfgs])
        nb = _sz(0)
        _call("lbm_batch_workspace_bytes", self.params, n, ctypes.byref(nb))
        self.device = torch.device(device)
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        h = _vp()
        st = torch.cuda.current_stream(self.device).cuda_stream
        _call("lbm_batch_create", self.params, n, _vp(ptr), nb.value, _vp(st), ctypes.byref(h))
        self.h = h.value

    def init_droplets(self, run, droplets, rho_L, rho_V, W):
        arr = _droplet_array(droplets)
        _call("lbm_batch_init_droplets", _vp(self.h), run, arr, len(droplets), rho_L, rho_V, W)

    def init_fields(self, run, rho, u):
        torch = _torch()
        r = torch.as_tensor(rho, dtype=torch.float64).to(self.device).contiguous()
        v = torch.as_tensor(u, dtype=torch.float64).to(self.device).contiguous()
        _call("lbm_batch_init_fields", _vp(self.h), run, _vp(r.data_ptr()), _vp(v.data_ptr()))
        torch.cuda.synchronize(self.device)

    def step(self, n, graph_steps=0):
        _call("lbm_batch_step", _vp(self.h), int(n), int(graph_steps))

    def read_populations(self, run):
        torch = _torch()
        c = self.cfgs[run]
        f = torch.empty((Q, c["nx"] * c["ny"] * c["nz"]), dtype=torch.float64, device=self.device)
        _call("lbm_batch_read_populations", _vp(self.h), run, _vp(f.data_ptr()))
        return f

    def read_fields(self, run):
        torch = _torch()
        c = self.cfgs[run]
        N = c["nx"] * c["ny"] * c["nz"]
        rho = torch.empty(N, dtype=torch.float64, device=self.device)
        u = torch.empty((3, N), dtype=torch.float64, device=self.device)
        p = torch.empty(N, dtype=torch.float64, device=self.device)
        _call("lbm_batch_read_fields", _vp(self.h), run, _vp(rho.data_ptr()), _vp(u.data_ptr()), _vp(p.data_ptr()))
        return {"rho": rho, "u": u, "p": p}

    def diagnostics(self, run, center=None, r_in=0.0, r_out=0.0):
        """Diagnostics of one run, as Lattice.diagnostics gives them."""
        req = _diag_request(center, r_in, r_out)
        d = LbmDiag()
        st = lib().lbm_batch_diagnostics(_vp(self.h), int(run), ctypes.byref(req) if req is not None else None,
                                         ctypes.byref(d))
        if st not in (0, -4):
            check(st, "lbm_batch_diagnostics")
        return _diag_dict(st, d)

    def status(self):
        """Per-run status codes (0 ok, -4 non-finite populations)."""
        n = lib().lbm_batch_runs(_vp(self.h))
        arr = (_i32 * n)()
        st = lib().lbm_batch_status(_vp(self.h), arr)
        if st not in (0, -4):
            check(st, "lbm_batch_status")
        return [int(v) for v in arr]

    @property
    def runs(self):
        return lib().lbm_batch_runs(_vp(self.h))

    def autotune(self, trials=3):
        b = _i32(0)
        _call("lbm_batch_autotune", _vp(self.h), int(trials), ctypes.byref(b))
        return b.value

    def set_blocks(self, blocks):
        _call("lbm_batch_set_blocks", _vp(self.h), int(blocks))

    def set_item_nodes(self, n):
        _call("lbm_batch_set_item_nodes", _vp(self.h), int(n))
        return self

    def tuning(self):
        """(step mode name, nodes per work item, grid blocks)."""
        m, it, bl = _i32(0), _i32(0), _i32(0)
        _call("lbm_batch_get_tuning", _vp(self.h), ctypes.byref(m), ctypes.byref(it), ctypes.byref(bl))
        return {v: k for k, v in STEP_MODES.items()}[m.value], it.value, bl.value

    def set_step_mode(self, mode):
        """mode: "fused", "pairs" or "split"."""
        _call("lbm_batch_set_step_mode", _vp(self.h), STEP_MODES[mode])
        return self

    def set_store_policy(self, policy):
        """Split step's population stores: "auto", "cached" or "stream"."""
        _call("lbm_batch_set_store_policy", _vp(self.h), STORE_POLICIES[policy])
        return self

    def step_mode(self):
        m = _i32(0)
        _call("lbm_batch_get_step_mode", _vp(self.h), ctypes.byref(m))
        return {v: k for k, v in STEP_MODES.items()}[m.value]

    def kernel_time(self):
        ms = ctypes.c_double(0)
        n = _i64(0)
        _call("lbm_batch_kernel_time", _vp(self.h), ctypes.byref(ms), ctypes.byref(n))
        return ms.value, n.value

    @property
    def nodes(self):
        return lib().lbm_batch_nodes(_vp(self.h))

    def close(self):
        if getattr(self, "h", None):
            _call("lbm_batch_destroy", _vp(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def storage_bytes(storage: str) -> int:
    return {"f64": 8, "f32": 4, "f16s": 2, "f16n": 2}[storage]


def planes(storage: str) -> int:
    """Values per node of a population array: 19 directions, plus the
    reference density of F16N."""
    return 20 if storage == "f16n" else 19


def population_bytes(storage: str, n: int) -> int:
    """Bytes of one population buffer of n nodes (the raw state without the
    step counter): the planes, then F16N's 16-byte rounding seed."""
    return planes(storage) * n * storage_bytes(storage) + (16 if storage == "f16n" else 0)


def algorithmic_bytes_per_node(storage: str) -> int:
    """19 population reads + 19 writes per lattice update (F16N: 20 + 20,
    with the reference densities)."""
    return 2 * planes(storage) * storage_bytes(storage)
