"""Host checks of the binary16 storage emulation (``tests/f16s_format.py``)
that the GPU tests of F16S and F16N compare the library against: the pull
layout maps, the toward-zero conversion, the stochastic rounding of the F16N
step and the FP64 write path.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest

from tests import f16s_format as fmt


@pytest.mark.parametrize("wall_z", [0, 1])
def test_pull_layout_maps_invert_each_other(wall_z):
    cfg = dict(nx=6, ny=5, nz=4, wall_z=wall_z)
    h = np.random.default_rng(3).normal(size=(19, 120))
    assert np.array_equal(fmt.stored(fmt.pulled(h, cfg), cfg), h)
    assert np.array_equal(fmt.pulled(fmt.stored(h, cfg), cfg), h)
    # every stored value has exactly one puller, and pulls stay on the lattice
    pul = fmt.puller_index(cfg)
    assert pul.min() >= 0 and pul.max() < 120


def test_pull_layout_bounces_back_at_walls():
    """A value leaving through a wall is pulled by its own node, in the
    opposite direction: with walls, stored(f)[a][x] = f[opp(a)][x] there."""
    from oracle import moments
    cfg = dict(nx=4, ny=4, nz=3, wall_z=1)
    f = np.arange(19 * 48, dtype=np.float64).reshape(19, 48)
    st = fmt.stored(f, cfg)
    for a, (ex, ey, ez) in enumerate(moments.VELOCITIES):
        if ez < 0:  # leaves through the bottom wall from z = 0
            assert np.array_equal(st[a][:16], f[moments.opposite(a)][:16])
        if ez > 0:  # through the top wall from z = nz - 1
            assert np.array_equal(st[a][32:], f[moments.opposite(a)][32:])


def _rtz_exact(x):
    """binary16 toward zero of one FP32 value, from the exact rational value."""
    q = Fraction(float(x))
    if q == 0:
        return np.float16(0.0)
    s, q = (-1 if q < 0 else 1), abs(q)
    e = -14
    while e < 15 and q >= Fraction(2) ** (e + 1):
        e += 1
    if q >= Fraction(65504):
        return np.float16(s * 65504.0)
    step = Fraction(2) ** (e - 10)  # normal and subnormal spacing (e = -14 below 2^-14)
    return np.float16(s * float((q // step) * step))


def test_toward_zero_conversion_matches_exact():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(scale=s, size=300) for s in (1e-6, 1e-3, 1.0, 300.0, 3e4)]).astype(np.float32)
    x = np.concatenate([x, np.array([0.0, 65504.0, 65519.99, 70000.0, -70000.0, 2.0 ** -14, 2.0 ** -24],
                                    dtype=np.float32)])
    got = fmt.f16_rtz(x)
    want = np.array([_rtz_exact(v) for v in x])
    assert np.array_equal(got.view(np.uint16), want.view(np.uint16))


def test_dither_is_uniform_13_bit():
    r = np.concatenate([fmt.dither(seed, np.arange(4096), a) for seed in range(4) for a in range(19)])
    assert r.min() == 0 and r.max() == 8191
    counts = np.bincount((r >> 9).astype(np.int64), minlength=16)  # 16 bins
    assert np.all(np.abs(counts / counts.mean() - 1) < 0.05)
    # the dithers change from step to step at a fixed node and direction
    per_step = np.array([fmt.dither(seed, np.array([77]), 5)[0] for seed in range(64)])
    assert len(np.unique(per_step)) > 50


@pytest.mark.parametrize("frac", [0.1, 0.3, 0.5, 0.9])
def test_stochastic_rounding_is_unbiased(frac):
    """Over the dithers of many nodes, a value a fraction `frac` of a binary16
    unit above a representable value rounds up with that probability, and the
    mean stored value equals it; nearest rounding would move it to a
    neighbour."""
    n = 200000
    base = 1.0 + 37 * 2.0 ** -10
    x = np.full(n, base + frac * 2.0 ** -10)
    rt = np.zeros((19, n), dtype=np.float16)
    cfg = dict(f16_exp=0)
    for a in (0, 7, 18):
        f = np.zeros((19, n))
        f[a] = x
        h = fmt.encode_n_sr(f, rt, cfg, seed=11)[a].astype(np.float64)
        assert set(np.unique(h)) <= {base, base + 2.0 ** -10}
        assert abs((h.mean() - base) / 2.0 ** -10 - frac) < 0.01


def test_write_path_rounds_once_to_binary16():
    """encode_n (the host write) takes the FP64 difference and rounds it once:
    at a value just below a binary16 midpoint it rounds down, where rounding
    through FP32 first would land on the midpoint and round to even (up)."""
    cfg = dict(f16_exp=0)
    lo, hi = 1.0 + 2.0 ** -10, 1.0 + 2.0 ** -9  # odd and even binary16 neighbours
    mid = 0.5 * (lo + hi)
    f = np.zeros((19, 1))
    f[0, 0] = mid - 2.0 ** -40  # rounds to the midpoint in FP32
    rt = np.zeros(1, dtype=np.float16)
    assert float(np.float32(f[0, 0])) == mid
    assert float(np.float32(f[0, 0]).astype(np.float16)) == hi  # the FP32 route: tie, to even
    assert float(fmt.encode_n(f, rt, cfg)[0, 0]) == lo  # one rounding: down


def test_decode_is_exact_sum():
    cfg = dict(f16_exp=12)
    rng = np.random.default_rng(9)
    h = rng.normal(scale=100, size=(19, 50)).astype(np.float16)
    rt = (rng.random(50) * 0.4 + 0.01).astype(np.float16)
    got = fmt.decode_n(h, rt, cfg)
    for a in (0, 3, 11):
        for i in (0, 17, 49):
            want = Fraction(float(h[a, i])) * Fraction(2) ** -12 + Fraction(float(fmt.W_CLASS[a])) * Fraction(float(rt[i]))
            assert abs(Fraction(float(got[a, i])) - want) <= abs(want) * Fraction(2) ** -52
