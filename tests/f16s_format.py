"""Host emulation of the shifted binary16 population storage (F16S), used by
the GPU tests to separate the format's rounding from the kernel's arithmetic.

The stored value of a population fbar_a is h = (v - shift_a) 2^e rounded once
(nearest even) to binary16, with v = fbar_a rounded to FP32 and
shift_a = w_a rho_ref rounded to FP32 (w = 1/3, 1/18, 1/36 by velocity
class).  Loading gives h 2^-e + shift_a rounded once to FP32.  The exactness
of this emulation against the library is pinned by
``test_f16_storage_format_round_trip``.  No lattice Boltzmann arithmetic
lives here.
"""
import numpy as np

W_CLASS = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _shift(cfg):
    return (W_CLASS * cfg["rho_ref"]).astype(np.float32).astype(np.float64)[:, None]


def encode(f, cfg):
    """binary16 values h of the FP64 populations f (shape (19, N))."""
    v = np.asarray(f, dtype=np.float64).astype(np.float32).astype(np.float64)
    return ((v - _shift(cfg)) * 2.0 ** cfg["f16_exp"]).astype(np.float16)


def decode(h, cfg):
    return (h.astype(np.float64) / 2.0 ** cfg["f16_exp"] + _shift(cfg)).astype(np.float32).astype(np.float64)


def round_trip(f, cfg):
    """What storing f and loading it back gives."""
    return decode(encode(f, cfg), cfg)


def ordered_bits(h):
    """binary16 values as integers ordered like the reals (adjacent
    representable values differ by 1; +0 and -0 both map to 0)."""
    b = h.view(np.uint16).astype(np.int64)
    return np.where(b & 0x8000, -(b & 0x7FFF), b)
