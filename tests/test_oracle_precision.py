"""Pins for the reference bfloat16 rounding (CPU only)."""
import numpy as np

from oracle.precision import bf16_bits_to_f64, to_bf16_bits


def test_exact_values_pass_through():
    vals = np.array([0.0, 1.0, -2.0, 0.5, 3.0, 1.0 + 2.0 ** -7, 65280.0, 2.0 ** -100])
    np.testing.assert_array_equal(bf16_bits_to_f64(to_bf16_bits(vals)), vals)


def test_ties_round_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: even mantissa (1.0) wins
    assert bf16_bits_to_f64(to_bf16_bits(np.array([1.0 + 2.0 ** -8])))[0] == 1.0
    # 1 + 3*2^-8 is halfway between 1+2^-7 (odd) and 1+2^-6 (even): rounds up
    assert bf16_bits_to_f64(to_bf16_bits(np.array([1.0 + 3 * 2.0 ** -8])))[0] == 1.0 + 2.0 ** -6
    assert bf16_bits_to_f64(to_bf16_bits(np.array([1.0 + 1.5 * 2.0 ** -8])))[0] == 1.0 + 2.0 ** -7


def test_relative_error_bound():
    x = np.random.default_rng(0).lognormal(0.0, 3.0, size=100000) * np.sign(
        np.random.default_rng(1).normal(size=100000))
    y = bf16_bits_to_f64(to_bf16_bits(x))
    # 8 significand bits: unit roundoff 2^-8
    assert np.max(np.abs(y - x) / np.abs(x)) <= 2.0 ** -8 * (1 + 1e-6)
    assert np.isnan(bf16_bits_to_f64(to_bf16_bits(np.array([np.nan])))[0])
