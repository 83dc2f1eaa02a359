"""Reference roundings for the reduced-precision copies (oracle; test infrastructure only).

f64 -> f32 is IEEE round-to-nearest-even (numpy's astype); f32 -> bfloat16 keeps the
upper 16 bits of the f32 pattern after round-to-nearest-even on the lower 16
(ties to even), NaN kept quiet.  Returned as raw uint16 bit patterns and as the
f64 values they represent.

Pins (tests/test_oracle_precision.py): exactly representable values pass through,
halfway cases round to even, the relative error is at most 2^-8 (8 significand bits).
"""
import numpy as np


def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def to_bf16_bits(x):
    f = to_f32(x)
    u = f.view(np.uint32).astype(np.uint64)
    is_special = (u & np.uint64(0x7F800000)) == np.uint64(0x7F800000)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    rounded = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) & np.uint64(0xFFFF)
    quiet = np.where((u & np.uint64(0xFFFF)) != 0, np.uint64(0x40), np.uint64(0))
    special = ((u >> np.uint64(16)) | quiet) & np.uint64(0xFFFF)
    return np.where(is_special, special, rounded).astype(np.uint16)


def bf16_bits_to_f64(bits):
    u = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)
