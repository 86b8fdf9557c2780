"""Pins of the oracle's storage-format rounding against library conversions."""
import numpy as np
import torch

from oracle import quantize as Q


def _samples():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(200000) * rng.choice([1e-6, 1e-3, 1.0, 30.0, 400.0, 1e5], 200000)
    special = [0.0, -0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -11,
               1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65504.0, 3.4e38]
    return np.concatenate([x, special]).astype(np.float32)


def test_bf16_matches_torch_rne():
    x = _samples()
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(Q.bf16_bits(x), want)
    assert np.array_equal(Q.bf16_value(want), torch.from_numpy(x).to(torch.bfloat16).float().numpy())


def test_bf16_split_is_exact_to_16_bits():
    x = _samples()
    x = x[np.abs(x) < 1e30]
    hi, lo = Q.bf16_split(x)
    s = Q.bf16_value(hi).astype(np.float64) + Q.bf16_value(lo).astype(np.float64)
    rel = np.abs(s - x) / np.maximum(np.abs(x), 1e-30)
    assert rel.max() <= 2.0 ** -16


def test_e4m3_matches_torch_in_range():
    x = _samples()
    x = x[np.abs(x) <= 448.0]
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(Q.e4m3_encode(x), want)
    codes = np.arange(256, dtype=np.uint8)
    tv = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(tv), np.isnan(Q.e4m3_table()))
    ok = ~np.isnan(tv)
    assert np.array_equal(tv[ok], Q.e4m3_table()[ok])


def test_e4m3_saturates_and_rowscale_bounds():
    assert Q.e4m3_decode(Q.e4m3_encode(np.float32([1e6, -500.0, 449.0])))[0] == 448.0
    rng = np.random.default_rng(1)
    a = (rng.standard_normal((64, 300)) * rng.uniform(1e-3, 1e3, (64, 1))).astype(np.float32)
    a[5] = 0.0
    q, s = Q.fp8_rowscaled(a)
    v = s[:, None].astype(np.float64) * Q.e4m3_decode(q)
    # e4m3 has 3 mantissa bits: relative error <= 2^-4 above the subnormal range
    big = np.abs(a) >= s[:, None] * 2.0 ** -6
    assert np.all(np.abs(v - a)[big] <= 2.0 ** -4 * np.abs(a)[big] * (1 + 1e-6))
    assert np.all(np.abs(v - a)[~big] <= s[:, None].repeat(300, 1)[~big] * 2.0 ** -10 * (1 + 1e-6))
    assert np.all(v[5] == 0.0)
    assert np.all(np.max(np.abs(Q.e4m3_decode(q)), axis=1)[np.arange(64) != 5] == 448.0)
