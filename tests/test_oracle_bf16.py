"""Pins of the bfloat16 split emulation."""
import numpy as np
import torch

from oracle import bf16


def test_hi_matches_torch_rne_conversion():
    """torch's float32 -> bfloat16 conversion is round-to-nearest-even."""
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(20000).astype(np.float32),
                        (rng.standard_normal(2000) * 1e-30).astype(np.float32),
                        (rng.standard_normal(2000) * 1e30).astype(np.float32)])
    hi = bf16.bf16_rne_bits(a)
    t = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(hi, t)


def test_tie_cases_round_to_even():
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)       # bf16 spacing at 1
    half = np.float32(2.0 ** -8)
    vals = np.array([one, one + half, one + ulp + half, one + half + np.float32(2 ** -20)], dtype=np.float32)
    hi = bf16.bf16_rne_bits(vals)
    assert list(hi) == [0x3F80, 0x3F80, 0x3F82, 0x3F81]


def test_split_error_bound_and_exact_remainder():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(50000).astype(np.float32) * np.float32(3.7)
    hv, lv = bf16.split_values(a)
    err = np.abs(a.astype(np.float64) - hv.astype(np.float64) - lv.astype(np.float64))
    assert np.all(err <= 2.0 ** -16 * np.abs(a.astype(np.float64)))
    # a - hi is exact in FP32
    rem32 = (a - hv).astype(np.float32)
    assert np.array_equal(rem32.astype(np.float64), a.astype(np.float64) - hv.astype(np.float64))
