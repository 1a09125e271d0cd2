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
