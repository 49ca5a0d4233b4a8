"""Host emulation of the shifted binary16 population storage (F16S), used by
the GPU tests to separate the format's rounding from the kernel's arithmetic.

The stored value of a population fbar_a is h = (v - shift_a) 2^e rounded once
(nearest even) to binary16, with v = fbar_a rounded to FP32 and
shift_a = w_a rho_ref rounded to FP32 (w = 1/3, 1/18, 1/36 by velocity
class).  Loading gives h 2^-e + shift_a rounded once to FP32.  The exactness
of this emulation against the library is pinned by
``test_f16_storage_format_round_trip``.  No lattice Boltzmann arithmetic
lives here.

F16N (binary16 relative to the pulling node) stores every population
arriving at node x against the shift w_a rt(x), where rt(x) is a density
rounded to binary16 and kept beside the populations.  The value a stored
h means is w_a rt(x) + h 2^-e exactly (the library's step works on the
deviations h 2^-e, which binary16 gives exactly in FP32); reading it back
in FP64 rounds the product and the sum once each.  Writing FP64 populations
takes the product and the difference in FP64 (each rounded once) and rounds
the scaled result once to binary16.  The library takes for rt(x) the density that x had
at the step that wrote the state.

The F16N step rounds its stores stochastically: the FP32 value gets a 13-bit
dither added to its bits and is truncated toward zero to binary16.  The
dither hashes the step's seed (kept after the planes, zero after a write,
one more every step), the index of the node whose post-collision value is
stored and the direction; ``encode_n_sr`` reproduces it bit for bit from the
same FP32 value.
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


def ref_bits(rho):
    """binary16 reference densities rt of FP64 (or FP32) densities, as the
    library rounds its FP32 density."""
    return np.asarray(rho, dtype=np.float64).astype(np.float32).astype(np.float16)


def _shift_n(rt):
    """FP64 shifts w_a rt (19, N) of binary16 references rt: shape (N,), one
    per node, or (19, N), one per stored value (each product rounded once)."""
    r = rt.astype(np.float64)
    return W_CLASS[:, None] * (r if r.ndim == 2 else r[None, :])


def encode_n(f, rt, cfg):
    """binary16 values h of FP64 populations f (19, N), each against the
    reference rt of the node that pulls it: (f - w_a rt) 2^e in FP64, rounded
    once to binary16."""
    d = (np.asarray(f, dtype=np.float64) - _shift_n(rt)) * 2.0 ** cfg["f16_exp"]
    return d.astype(np.float16)


def decode_n(h, rt, cfg):
    """FP64 values w_a rt + h 2^-e of populations h (19, N) stored against
    the references rt of the nodes that pull them."""
    return h.astype(np.float64) * 2.0 ** -cfg["f16_exp"] + _shift_n(rt)


def round_trip_n(f, rho_prev, cfg):
    """What storing the states f (19, N) (f_a(x): what node x pulls) against
    the references of the densities rho_prev (N) and loading them gives."""
    rt = ref_bits(rho_prev)
    return decode_n(encode_n(f, rt, cfg), rt, cfg)


# --- stochastic rounding of the F16N step ---------------------------------
_M = 0xFFFFFFFF


def mix32(h):
    """32-bit integer finaliser (xorshift-multiply rounds, the constants of
    C. Wellons' lowbias32), elementwise on unsigned integers."""
    h = np.asarray(h, dtype=np.uint64) & _M
    h ^= h >> 16
    h = (h * 0x7FEB352D) & _M
    h ^= h >> 15
    h = (h * 0x846CA68B) & _M
    h ^= h >> 16
    return h


def dither(seed, src, a):
    """13-bit dithers of direction a for the values of source nodes src."""
    key = mix32((int(seed) + 0x9E3779B9) & _M)
    nh = mix32(np.asarray(src, dtype=np.uint64) ^ key)
    return ((nh + ((a * 0x9E3779B9) & _M)) & _M) >> 19


def f16_rtz(y):
    """binary16 values of FP32 y rounded toward zero (finite values beyond
    the binary16 range give the largest finite one)."""
    y = np.asarray(y, dtype=np.float32)
    b = y.view(np.uint32)
    normal = (b & 0x7FFFFFFF) >= (113 << 23)  # |y| >= 2^-14
    t = np.where(normal, (b & 0xFFFFE000).view(np.float32),
                 (np.trunc(y.astype(np.float64) * 2.0 ** 24) * 2.0 ** -24).astype(np.float32))
    big = np.isfinite(t) & (np.abs(t) >= 65536.0)
    t = np.where(big, np.copysign(np.float32(65504.0), t), t)
    return t.astype(np.float16)


def encode_n_sr(f, rt, cfg, seed, src=None):
    """The F16N step's stores of post-collision values f (19, n) of source
    nodes src (default 0 .. n - 1), each against the reference rt (19, n) of
    the node that pulls it: (f - w_a rt) 2^e in FP64 rounded to FP32, then
    the dither of (seed, src, a) added to its bits and the sum truncated
    toward zero to binary16."""
    x = ((np.asarray(f, dtype=np.float64) - _shift_n(rt)) * 2.0 ** cfg["f16_exp"]).astype(np.float32)
    if src is None:
        src = np.arange(x.shape[1])
    r = np.stack([dither(seed, src, a) for a in range(x.shape[0])]).astype(np.uint32)
    y = ((x.view(np.uint32).astype(np.uint64) + r) & _M).astype(np.uint32).view(np.float32)
    return f16_rtz(y)


# --- pull layout -------------------------------------------------------------
def _grid(cfg):
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return nx, ny, nz, x, y, z, ((z * ny + y) * nx + x).reshape(-1)


def puller_index(cfg):
    """(19, N) index of the node that pulls the value stored at (a, x'):
    x' + e_a (periodic), or x' itself where that lies beyond a wall."""
    from oracle import moments
    nx, ny, nz, x, y, z, own = _grid(cfg)
    out = np.empty((19, nx * ny * nz), dtype=np.int64)
    for a, (ex, ey, ez) in enumerate(moments.VELOCITIES):
        zz = z + ez
        beyond = (((zz < 0) | (zz >= nz)) if cfg.get("wall_z", 0) else np.zeros_like(zz, dtype=bool)).reshape(-1)
        d = (((zz % nz) * ny + (y + ey) % ny) * nx + (x + ex) % nx).reshape(-1)
        out[a] = np.where(beyond, own, d)
    return out


def pulled(h, cfg):
    """Stored values (19, N) in the order of the nodes that pull them:
    element (a, x) is what x pulls in direction a, h[a][x - e_a], or
    h[opp(a)][x] where x - e_a lies beyond a wall."""
    from oracle import moments
    nx, ny, nz, x, y, z, own = _grid(cfg)
    out = np.empty_like(h)
    for a, (ex, ey, ez) in enumerate(moments.VELOCITIES):
        zz = z - ez
        beyond = (((zz < 0) | (zz >= nz)) if cfg.get("wall_z", 0) else np.zeros_like(zz, dtype=bool)).reshape(-1)
        s = (((zz % nz) * ny + (y - ey) % ny) * nx + (x - ex) % nx).reshape(-1)
        out[a] = np.where(beyond, h[moments.opposite(a)][own], h[a][s])
    return out


def stored(fp, cfg):
    """Inverse of ``pulled``: the post-collision value of direction a at node
    x' (what its puller receives) from states fp (19, N) in pulled order."""
    from oracle import moments
    nx, ny, nz, x, y, z, own = _grid(cfg)
    out = np.empty_like(fp)
    for a, (ex, ey, ez) in enumerate(moments.VELOCITIES):
        zz = z + ez
        beyond = (((zz < 0) | (zz >= nz)) if cfg.get("wall_z", 0) else np.zeros_like(zz, dtype=bool)).reshape(-1)
        d = (((zz % nz) * ny + (y + ey) % ny) * nx + (x + ex) % nx).reshape(-1)
        out[a] = np.where(beyond, fp[moments.opposite(a)][own], fp[a][d])
    return out


def round_trip_n_sr(f, rho_prev, cfg, seed):
    """What the F16N step stores of the states f (19, N) (pulled order, after
    collision and streaming) and what the next step loads back: each value
    rounded stochastically with the step's seed against the reference of its
    puller, the binary16 density rho_prev had there."""
    rt = ref_bits(rho_prev)
    h = encode_n_sr(stored(f, cfg), rt[puller_index(cfg)], cfg, seed)
    return decode_n(pulled(h, cfg), rt, cfg)
