"""The e4m3 reference encoder against the format's definition (CPU)."""
import numpy as np

from tests import fp8_format as f8


def test_every_finite_code_round_trips():
    codes = np.arange(256)
    vals = f8.decode(codes)
    finite = ~np.isnan(vals)
    assert finite.sum() == 254                      # two NaN codes, no infinities
    assert np.nanmax(vals) == 448.0 and np.nanmin(vals) == -448.0
    assert f8.decode(1) == 2.0 ** -9                # smallest subnormal
    back = f8.round_e4m3(vals[finite])
    assert np.array_equal(back, vals[finite])


def test_midpoints_round_to_even_mantissa():
    pos = np.sort(f8.decode(np.arange(0, 127)))     # 0 .. 448 (code 127 is NaN)
    mids = 0.5 * (pos[:-1] + pos[1:])
    got = f8.round_e4m3(mids)
    codes_lo = np.arange(0, 126)
    # the even neighbour (last mantissa bit clear) wins each tie
    want = np.where(codes_lo % 2 == 0, pos[:-1], pos[1:])
    assert np.array_equal(got, want)


def test_nearest_value_brute_force():
    rng = np.random.default_rng(0)
    x = rng.uniform(-448, 448, 20000) * np.exp2(rng.integers(-14, 1, 20000))
    table = f8.decode(np.arange(256))
    table = table[~np.isnan(table)]
    got = f8.round_e4m3(x)
    dist = np.abs(x[:, None] - table[None, :])
    best = np.min(dist, axis=1)
    assert np.allclose(np.abs(got - x), best, rtol=0, atol=0)


def test_scales_are_minimal_powers_of_two():
    amax = np.array([448.0, 448.0001, 1.0, 3.5, 896.0, 1e-30])
    s = f8.pow2_scale(amax)
    assert np.all(amax / s <= 448.0)
    assert np.all(amax / (s / 2) > 448.0)
    assert f8.pow2_scale(0.0) == 1.0
    # the floor: blocks below 448 * 2^-126 keep the scale 2^-126 and still fit
    tiny = np.array([1e-40, 448.0 * 2.0 ** -126, 448.0 * 2.0 ** -125])
    st = f8.pow2_scale(tiny)
    assert list(st) == [2.0 ** -126, 2.0 ** -126, 2.0 ** -125]
    assert np.all(tiny / st <= 448.0)
