"""ctypes binding of ``include/mrt_probe.h``: the HBM data-movement probes
(argument marshalling only; the kernels are in ``lib/libmrtprobe.so``)."""
from __future__ import annotations

import ctypes
import os

from .binding import LbmError

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libmrtprobe.so")

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t
SIGNATURES = {
    "lbm_probe_copy": (_i32, [_vp, _vp, _sz, _i32, _i32, _vp]),
    "lbm_probe_stream19": (_i32, [_vp, _vp, _sz, _i32, _i32, _i32, _vp]),
    "lbm_probe_march19": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _vp]),
    "lbm_probe_last_error": (ctypes.c_char_p, []),
}
_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"probe library not built: {LIB_PATH} missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise LbmError(st, name, lib().lbm_probe_last_error().decode(errors="replace"))


def lbm_probe_copy(src, dst, nbytes, streaming_stores, blocks, stream):
    _call("lbm_probe_copy", _vp(src), _vp(dst), nbytes, int(streaming_stores), int(blocks), _vp(stream))


def lbm_probe_stream19(src, dst, plane_bytes, group_bytes, streaming_stores, blocks, stream):
    _call("lbm_probe_stream19", _vp(src), _vp(dst), plane_bytes, int(group_bytes), int(streaming_stores),
          int(blocks), _vp(stream))


def lbm_probe_march19(src, dst, nx_groups, ny, nz, group_bytes, tx, ty, cz, streaming_stores, stream):
    _call("lbm_probe_march19", _vp(src), _vp(dst), int(nx_groups), int(ny), int(nz), int(group_bytes),
          int(tx), int(ty), int(cz), int(streaming_stores), _vp(stream))
