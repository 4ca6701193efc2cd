"""Pins of the oracle's bit-plane truncation (Sec. 4.2, Eq. (12); Sec. 3.7).

Expected values come from the paper's worked example, from the IEEE-754
definition of the exponent, and from an independent frexp/ldexp formulation
of "keep m mantissa bits, round toward zero" -- never from the oracle itself.
"""
import json
import math
import os
import struct

import numpy as np
import pytest

from oracle import qcz_oracle as oq

GOLD = os.path.join(os.path.dirname(__file__), "golden")
DELTAS = [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]


def f2b(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def b2f(b):
    return struct.unpack("<d", struct.pack("<Q", b))[0]


def chop_mantissa(x, m):
    """|x| cut toward zero to m fraction bits, sign kept (frexp/ldexp form)."""
    if x == 0.0:
        return x
    f, e = math.frexp(abs(x))            # |x| = f * 2^e, f in [0.5, 1)
    scaled = math.ldexp(f, m + 1)        # 1.xxx with m fraction bits above the point
    return math.copysign(math.ldexp(math.floor(scaled), e - m - 1), x)


def test_sigbits_example_from_paper():
    g = json.load(open(os.path.join(GOLD, "sigbits_example.json")))
    assert oq.exp_of(g["eps"]) == g["EXP"]
    level = DELTAS.index(g["eps"])
    assert oq.sig_bits(level) == g["bit_count_sign_exp_binary64"] - g["EXP"]


@pytest.mark.parametrize("level,expected_m", [(1, 17), (2, 14), (3, 10), (4, 7), (5, 4)])
def test_mantissa_bits_per_level(level, expected_m):
    # EXP(delta) = floor(log2(delta)) for these non-powers of two
    assert oq.exp_of(DELTAS[level]) == math.floor(math.log2(DELTAS[level]))
    assert oq.sig_bits(level) == 12 + expected_m
    assert 2.0 ** -expected_m <= DELTAS[level] < 2.0 ** -(expected_m - 1)


def test_paper_worked_example_both_readings():
    g = json.load(open(os.path.join(GOLD, "paper_truncation_example.json")))
    v = g["value"]
    # The example is binary32; the same value in binary64 keeps the same
    # leading bits.  Eq. (12) at eps = 0.01 keeps 7 mantissa bits:
    level = DELTAS.index(g["eps"])
    t = oq.truncate(np.array([v]), level)[0]
    assert t == 3.984375 == chop_mantissa(v, 7)
    # The printed result keeps 15 binary32 bits = 9 sign/exponent + 6 mantissa:
    K_printed = 12 + (g["paper_kept_leading_bits"] - 9)
    t_printed = b2f(oq.truncate_bits(f2b(v), K_printed))
    assert t_printed == g["paper_decompressed"]
    assert abs((v - t_printed) / v - g["paper_relative_error"]) < 5e-7
    # Only the Eq. (12) reading honours the bound for every value of that binade
    worst = (1.0156249 - chop_mantissa(1.0156249, 6)) / 1.0156249
    assert worst > g["eps"]
    assert (1.0156249 - chop_mantissa(1.0156249, 7)) / 1.0156249 < g["eps"]


def _sample_doubles(rng, count):
    # every exponent of the normal range x a spread of mantissas, both signs
    e = rng.integers(-1021, 1023, size=count)
    f = rng.uniform(0.5, 1.0, size=count)
    s = np.where(rng.random(count) < 0.5, -1.0, 1.0)
    return s * np.ldexp(f, e)


@pytest.mark.parametrize("level", range(1, 6))
def test_truncation_matches_independent_definition(level):
    rng = np.random.default_rng(100 + level)
    xs = _sample_doubles(rng, 4000)
    m = 12 - oq.exp_of(DELTAS[level]) - 12
    ts = oq.truncate(xs, level)
    for x, t in zip(xs, ts):
        assert t == chop_mantissa(float(x), m)


@pytest.mark.parametrize("level", range(0, 6))
def test_truncation_invariants(level):
    rng = np.random.default_rng(7 + level)
    xs = np.concatenate([_sample_doubles(rng, 3000), [0.0, -0.0, 1.0, -1.0, 0.5, 2.0 ** -20]])
    ts = oq.truncate(xs, level)
    delta = DELTAS[level]
    ebound = 0.0 if level == 0 else 2.0 ** oq.exp_of(delta)
    for x, t in zip(xs, ts):
        x, t = float(x), float(t)
        assert math.copysign(1, t) == math.copysign(1, x)          # sign kept, -0 kept
        if x == 0.0:
            assert f2b(t) == f2b(x)
            continue
        rel = (abs(x) - abs(t)) / abs(x)
        assert 0.0 <= rel                                            # toward zero: |D'| <= |D|
        assert rel < ebound or (level == 0 and rel == 0.0)           # strict form of (|D(1-d)|, |D|]
        assert ebound <= delta
        assert oq.truncate(np.array([t]), level)[0] == t              # idempotent
        assert oq.truncate(np.array([-x]), level)[0] == -t            # odd
    for lo in range(level, 6):                                       # masks nest
        t2 = oq.truncate(oq.truncate(xs, level), lo)
        assert np.array_equal(t2.view(np.uint64), oq.truncate(xs, lo).view(np.uint64))


def test_every_exponent_and_top_mantissa_patterns():
    # exhaustive over all 2046 normal exponents x the 256 top-mantissa patterns
    level = 3
    m = 10
    exps = np.arange(1, 2047, dtype=np.uint64)
    tops = np.arange(256, dtype=np.uint64)
    bits = ((exps[:, None] << np.uint64(52)) | (tops[None, :] << np.uint64(44)) | np.uint64(0x5A5A5A5A5A5)).ravel()
    xs = bits.view(np.float64)
    ts = oq.truncate(xs, level)
    expect = bits & ~np.uint64((1 << (52 - m)) - 1)
    assert np.array_equal(ts.view(np.uint64), expect)
