"""Pins of the oracle's chunk codec (Solution C of Sec. 4.2 + the project's
lossless stage).  Expected bytes of small chunks are derived by hand in
``golden/chunks_small.json``; larger chunks are checked through properties
that any correct codec has (decode(encode(x)) equals the truncation of x,
independently of stream order, Sec. 4.2 on Solutions C and D)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import qcz_oracle as oq

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def chop(xs, level):
    """Independent truncation: keep m = -EXP(delta) fraction bits (frexp form)."""
    if level == 0:
        return np.array(xs, dtype=np.float64)
    m = -math.floor(math.log2([0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1][level]))
    out = []
    for x in np.asarray(xs, dtype=np.float64):
        x = float(x)
        if x == 0.0:
            out.append(x)
            continue
        f, e = math.frexp(abs(x))
        out.append(math.copysign(math.ldexp(math.floor(math.ldexp(f, m + 1)), e - m - 1), x))
    return np.array(out)


def same_bits(a, b):
    return np.array_equal(np.asarray(a, dtype=np.float64).view(np.uint64),
                          np.asarray(b, dtype=np.float64).view(np.uint64))


def test_golden_small_chunks():
    g = json.load(open(os.path.join(GOLD, "chunks_small.json")))
    for case in g["cases"]:
        expect = bytes.fromhex(case["hex"].replace(" ", ""))
        got = oq.encode_chunk(np.array(case["values"]), case["level"])
        assert got == expect, case["name"]
        dec = oq.decode_chunk(expect, len(case["values"]))
        assert same_bits(dec, chop(case["values"], case["level"]))


def chunk_family(rng, C, kind):
    if kind == "random":
        return rng.normal(size=C) * 2.0 ** -12
    if kind == "zeros":
        return np.zeros(C)
    if kind == "const2":
        return np.tile([0.125, -0.3], C // 2)
    if kind == "sparse":
        x = np.zeros(C)
        idx = rng.choice(C, size=max(1, C // 64), replace=False)
        x[idx] = rng.normal(size=idx.size)
        return x
    if kind == "halfzero":
        x = rng.normal(size=C)
        x[1::2] = 0.0
        return x
    if kind == "signed_zero":
        x = rng.normal(size=C)
        x[rng.random(C) < 0.3] = -0.0
        return x
    if kind == "wide_exponents":
        return rng.normal(size=C) * np.ldexp(1.0, rng.integers(-900, 900, size=C))
    if kind == "repeats":
        return np.repeat(rng.normal(size=C // 8), 8)
    raise ValueError(kind)


FAMILIES = ["random", "zeros", "const2", "sparse", "halfzero", "signed_zero", "wide_exponents", "repeats"]


@pytest.mark.parametrize("C", [8, 64, 512, 2048])
@pytest.mark.parametrize("level", range(6))
def test_roundtrip_equals_truncation(C, level):
    rng = np.random.default_rng(C * 10 + level)
    for kind in FAMILIES:
        x = chunk_family(rng, C, kind)
        blob = oq.encode_chunk(x, level)
        assert len(blob) <= oq.chunk_cap(C)
        dec = oq.decode_chunk(blob, C)
        assert same_bits(dec, chop(x, level)), (kind, C, level)
        # header carries the level and a valid mode
        hdr = int.from_bytes(blob[:4], "little")
        assert hdr >> 5 == 0 and (hdr & 3) in (0, 1, 2) and (hdr >> 2) & 7 == level


def test_subnormal_chunk_is_lossless():
    x = np.array([1.0, 2.0 ** -1070, 0.3, -0.7])
    blob = oq.encode_chunk(x, 3)
    assert (int.from_bytes(blob[:4], "little") >> 2) & 7 == 0
    assert same_bits(oq.decode_chunk(blob, 4), x)


def test_const2_sizes_and_mode():
    for C in (4, 64, 2048):
        blob = oq.encode_chunk(np.tile([0.25, -0.5], C // 2), 2)
        assert len(blob) == 20 and blob[0] & 3 == 1


def test_lossless_random_size_bounds():
    # random mantissas are incompressible: lossless codes cost 2 bits, repeated
    # sign/exponent bytes save at most 24 bits per value
    rng = np.random.default_rng(3)
    C = 2048
    x = rng.normal(size=C)
    blob = oq.encode_chunk(x, 0)
    assert 4 + C // 4 + C * 5 <= len(blob) <= 4 + C // 4 + C * 8


def test_lossy_size_matches_bitcount_model():
    # At 1e-4 (K = 26) a value costs 2 code bits + 26 - 8 L residual bits.
    # For values of one binade and random signs, L is 0 on a sign change
    # and 1 otherwise (identical sign/exponent byte, differing byte 1 is
    # almost sure for random mantissas).
    rng = np.random.default_rng(4)
    C = 2048
    signs = np.where(rng.random(C) < 0.5, -1.0, 1.0)
    x = signs * rng.uniform(1.0, 1.999, size=C) * 2.0 ** -10
    blob = oq.encode_chunk(x, 2)
    flips = int(np.sum(signs[1:] != signs[:-1])) + 1      # first value differs from 0
    b = np.frombuffer(np.array(x).tobytes(), dtype=np.uint8).reshape(C, 8)[:, ::-1]
    same1 = np.r_[False, (b[1:, 1] == b[:-1, 1]) & (signs[1:] == signs[:-1])]
    same2 = same1 & np.r_[False, b[1:, 2] == b[:-1, 2]]
    n2, n3 = int(same1.sum()) - int(same2.sum()), int(same2.sum())
    bits = 26 * flips + 18 * (C - flips - n2 - n3) + 10 * n2 + 2 * n3
    assert len(blob) == 4 + C // 4 + (bits + 7) // 8


def test_order_independence_of_errors():
    # Sec. 4.2: Solution C and D (re/im reshuffled) give identical pointwise
    # errors because truncation does not depend on the order of the values.
    rng = np.random.default_rng(5)
    C = 512
    x = rng.normal(size=C) * 1e-3
    perm = np.r_[np.arange(0, C, 2), np.arange(1, C, 2)]
    for level in range(1, 6):
        a = oq.decode_chunk(oq.encode_chunk(x, level), C)
        b = oq.decode_chunk(oq.encode_chunk(x[perm], level), C)
        assert same_bits(a[perm], b)


def test_brute_force_tiny_chunks():
    vals = [0.0, -0.0, 1.0, -1.0, 0.75, 2.0 ** -30, 3.9921875]
    for combo in itertools.product(vals, repeat=4):
        x = np.array(combo)
        for level in (0, 2, 5):
            blob = oq.encode_chunk(x, level)
            assert same_bits(oq.decode_chunk(blob, 4), chop(x, level))


def test_decoder_rejects_malformed():
    rng = np.random.default_rng(6)
    x = rng.normal(size=512)
    blob = oq.encode_chunk(x, 1)
    with pytest.raises(ValueError):
        oq.decode_chunk(blob[:-3], 512)                  # truncated stream
    bad = bytearray(blob)
    bad[0] = (bad[0] & ~0x1C) | (7 << 2)                # level 7 does not exist
    with pytest.raises(ValueError):
        oq.decode_chunk(bytes(bad), 512)
    bad = bytearray(blob)
    bad[0] |= 3                                         # reserved mode
    with pytest.raises(ValueError):
        oq.decode_chunk(bytes(bad), 512)
    with pytest.raises(ValueError):
        oq.decode_chunk(blob + b"\0\0\0\0", 512)        # trailing garbage
