"""Host emulation of the shifted binary16 population storage (F16S), used by
the GPU tests to separate the format's rounding from the kernel's arithmetic.

The stored value of a population fbar_a is h = (v - shift_a) 2^e rounded once
(nearest even) to binary16, with v = fbar_a rounded to FP32 and
shift_a = w_a rho_ref rounded to FP32 (w = 1/3, 1/18, 1/36 by velocity
class).  Loading gives h 2^-e + shift_a rounded once to FP32.  The exactness
of this emulation against the library is pinned by
``test_f16_storage_format_round_trip``.  No lattice Boltzmann arithmetic
lives here.

F16N (binary16 relative to the pulling node) has the same rounding with a
shift per node: every population arriving at node x is stored against
shift_a = w_a rt(x) (one FP32 product), where rt(x) is a density rounded to
binary16 and kept beside the populations.  The library takes for rt(x) the
density that x had at the step that wrote the state.
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


W32 = W_CLASS.astype(np.float32)


def ref_bits(rho):
    """binary16 reference densities rt of FP64 (or FP32) densities, as the
    library rounds its FP32 density."""
    return np.asarray(rho, dtype=np.float64).astype(np.float32).astype(np.float16)


def node_shift(rt):
    """FP32 shifts w_a rt (shape (19, N)) of binary16 references rt: shape
    (N,), one per node, or (19, N), one per stored value."""
    r = rt.astype(np.float32)
    return W32[:, None] * (r if r.ndim == 2 else r[None, :])


def encode_n(f, rt, cfg):
    """binary16 values h of populations f (19, N), each against the
    reference rt of the node that pulls it: (v - shift) in FP32, scaled by
    2^e (exact), rounded to binary16."""
    v = np.asarray(f, dtype=np.float64).astype(np.float32)
    return ((v - node_shift(rt)) * np.float32(2.0 ** cfg["f16_exp"])).astype(np.float16)


def decode_n(h, rt, cfg):
    """FP64 values of populations h (19, N) stored against the references rt
    of the nodes that pull them."""
    v = h.astype(np.float32) * np.float32(2.0 ** -cfg["f16_exp"]) + node_shift(rt)
    return v.astype(np.float32).astype(np.float64)


def round_trip_n(f, rho_prev, cfg):
    """What storing the states f (19, N) (f_a(x): what node x pulls) against
    the references of the densities rho_prev (N) and loading them gives."""
    rt = ref_bits(rho_prev)
    return decode_n(encode_n(f, rt, cfg), rt, cfg)
