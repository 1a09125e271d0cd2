"""Exhaustive pins of the oracle's BF16 / E4M3FN rounding against torch's
conversions (library routine) and the formats' definitions (CPU only)."""
import numpy as np
import torch

from oracle import round_bf16, round_e4m3


def _all_bf16():
    codes = torch.arange(0, 1 << 16, dtype=torch.int32).to(torch.int16)
    return codes.view(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_codes_fixed_points():
    v = _all_bf16()
    fin = np.isfinite(v)
    assert np.array_equal(round_bf16(v[fin]), v[fin])


def test_bf16_midpoints_tie_to_even():
    v = np.sort(np.unique(_all_bf16()[np.isfinite(_all_bf16())]))
    v = v[(v > 0)]
    mid = (v[:-1] + v[1:]) / 2
    r = round_bf16(mid)
    # the even neighbour has a zero lowest mantissa bit
    lo_bits = torch.from_numpy(v[:-1].astype(np.float32)).view(torch.int32).numpy() >> 16
    even_is_lo = (lo_bits & 1) == 0
    assert np.array_equal(r, np.where(even_is_lo, v[:-1], v[1:]))


def test_bf16_matches_torch_on_random_float32():
    g = np.random.default_rng(1)
    x = (g.standard_normal(200000) * np.exp(g.uniform(-60, 60, 200000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(round_bf16(x.astype(np.float64)), ref)


def test_e4m3_codes_and_random():
    codes = torch.arange(0, 256, dtype=torch.int32).to(torch.uint8)
    v = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    fin = np.isfinite(v)
    assert fin.sum() == 254          # two NaN codes, no infinities
    assert np.array_equal(round_e4m3(v[fin]), v[fin])
    assert np.nanmax(v) == 448.0
    g = np.random.default_rng(2)
    x = (g.uniform(-440, 440, 100000) * np.exp(g.uniform(-12, 0, 100000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(round_e4m3(x.astype(np.float64)), ref)
    # saturation and the smallest subnormal
    assert round_e4m3(1e6) == 448.0 and round_e4m3(-500.0) == -448.0
    assert round_e4m3(2.0 ** -9) == 2.0 ** -9 and round_e4m3(2.0 ** -11) == 0.0


def _brute_margin(x, values):
    """Relative distance to the nearest midpoint of consecutive values (brute force)."""
    v = np.sort(np.unique(values))
    mid = (v[:-1] + v[1:]) / 2
    j = np.searchsorted(mid, x)
    lo = mid[np.clip(j - 1, 0, mid.size - 1)]
    hi = mid[np.clip(j, 0, mid.size - 1)]
    return np.minimum(np.abs(x - lo), np.abs(x - hi)) / np.abs(x)


def test_bf16_rounding_margin_against_code_enumeration():
    from oracle import bf16_rounding_margin
    v = _all_bf16()
    v = v[np.isfinite(v)]
    g = np.random.default_rng(3)
    x = np.concatenate([g.standard_normal(20000) * np.exp(g.uniform(-30, 30, 20000)),
                        g.uniform(-1, 1, 20000)])
    got = bf16_rounding_margin(x)
    ref = _brute_margin(x, v)
    normal = np.abs(x) >= 2.0 ** -126
    assert np.allclose(got[normal], ref[normal], rtol=1e-12, atol=0)
    assert (ref[normal] < 2.0 ** -12).sum() > 100
    # values on a boundary have margin 0; bfloat16 values sit half a spacing away
    mids = (v[(v > 0.5) & (v < 2)][:-1] + v[(v > 0.5) & (v < 2)][1:]) / 2
    assert np.all(bf16_rounding_margin(mids) == 0.0)
    # 1.0: the nearest boundary is 1 - 2^-9 (the spacing halves below 1); 1.5: 1.5 +- 2^-8
    assert bf16_rounding_margin(1.0) == 2.0 ** -9 and bf16_rounding_margin(1.5) == 2.0 ** -8 / 1.5


def test_bf16_rounding_margin_decides_like_rounding():
    """A perturbation below the margin never changes the bfloat16 rounding;
    one just beyond it in the right direction does."""
    from oracle import bf16_rounding_margin
    g = np.random.default_rng(4)
    x = g.uniform(0.01, 1.0, 50000)
    m = bf16_rounding_margin(x)
    for f in (0.999, -0.999):
        assert np.array_equal(round_bf16(x * (1 + f * m)), round_bf16(x))
    up = round_bf16(x * (1 + 1.001 * m)) != round_bf16(x)
    dn = round_bf16(x * (1 - 1.001 * m)) != round_bf16(x)
    assert np.all(up | dn)


def test_e4m3_rounding_margin_against_code_enumeration():
    from oracle import e4m3_rounding_margin
    codes = torch.arange(0, 256, dtype=torch.int32).to(torch.uint8)
    v = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    v = v[np.isfinite(v)]
    g = np.random.default_rng(5)
    x = g.uniform(-440, 440, 20000) * np.exp(g.uniform(-10, 0, 20000))
    got = e4m3_rounding_margin(x)
    ref = _brute_margin(x, v)
    inside = np.abs(x) < 448.0 - 16.0
    assert np.allclose(got[inside], ref[inside], rtol=1e-12, atol=0)
    assert e4m3_rounding_margin(500.0) == np.inf and e4m3_rounding_margin(1.0) == 2.0 ** -5
