"""Oracle pins of Solution B (Sec. 4.2): log-domain quantization of each value
(the IEEE-754 bit pattern of |x| as a piecewise-linear logarithm), prediction
from the previous nonzero value of the same part (real from real, imaginary
from imaginary), 16,384 symbols, Huffman codes.  Pinned by the pointwise
error bound, a closed-form stream (powers of two), an independent Python
decoder written from the stream layout, Huffman optimality against a heap
construction, and malformed streams."""
import heapq
import math
import struct

import numpy as np
import pytest

from oracle import qcz_oracle as oq

DELTA = [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]


def families(rng, C):
    f = {"normal": rng.normal(size=C), "huge": rng.normal(size=C) * 1e300, "tiny": rng.normal(size=C) * 1e-300,
         "smooth": np.repeat(np.cos(np.linspace(0, 3, C // 2)), 2) * 1e-3, "zeros": np.zeros(C),
         "negzeros": -np.zeros(C)}
    s = rng.normal(size=C)
    s[rng.random(C) < 0.7] = 0.0
    f["sparse"] = s
    ph = rng.uniform(0, 2 * np.pi, size=C // 2)
    f["phases"] = np.stack([np.cos(ph), np.sin(ph)], axis=1).reshape(-1) * 2.0 ** -17
    sp = rng.normal(size=C)
    sp[3] = 5e-324          # subnormal
    sp[10] = np.inf
    sp[11] = -np.inf
    sp[20] = 1.7976931348623157e308
    sp[21] = -0.0
    f["specials"] = sp
    return f


def test_bin_widths_are_the_largest_within_the_bound():
    for level in range(1, 6):
        t = 52 - oq.pred_width(level)
        assert 2.0 ** -(t + 1) <= DELTA[level] < 2.0 ** -t, level
    assert oq.pred_width(0) == -1


@pytest.mark.parametrize("C", [64, 256, 2048])
@pytest.mark.parametrize("level", range(1, 6))
def test_pointwise_bound_signs_and_specials(C, level):
    rng = np.random.default_rng(C + 7 * level)
    for name, x in families(rng, C).items():
        y = oq.decode_chunk(oq.encode_pred(x, level), C)
        fin = np.isfinite(x)
        assert np.all(np.abs(y[fin] - x[fin]) <= DELTA[level] * np.abs(x[fin])), name
        assert np.array_equal(np.signbit(y), np.signbit(x)), name
        assert np.array_equal(y[~fin], x[~fin]), name
        sub = (x != 0) & (np.abs(x) < 2.2250738585072014e-308)
        assert np.array_equal(y[sub], x[sub]), name   # subnormals are stored verbatim


def py_decode(b, C):
    """Solution B stream decoder written from the layout alone."""
    hdr = struct.unpack_from("<I", b, 0)[0]
    assert hdr & 3 == 3 and hdr >> 5 == 0
    w = 52 - {1: 16, 2: 13, 3: 9, 4: 6, 5: 3}[(hdr >> 2) & 7]
    A, NS = C // 2, C // 32
    cnt = struct.unpack_from("<16H", b, 4)
    sub = struct.unpack_from("<%dH" % NS, b, 36)
    o = 36 + 2 * NS
    nsym = sum(cnt)
    syms = struct.unpack_from("<%dH" % nsym, b, o)
    o = (o + 2 * nsym + 3) & ~3
    bits = int.from_bytes(b[o:o + 4 * ((sum(sub) + 31) // 32)], "little")
    o += 4 * ((sum(sub) + 31) // 32)
    table, code, idx = {}, 0, 0
    for ln in range(1, 17):              # canonical codes, (length, symbol) order
        for _ in range(cnt[ln - 1]):
            table[(ln, code)] = syms[idx]
            code += 1
            idx += 1
        code <<= 1
    pos, out_sym, out_sgn = 0, [], []
    for i in range(NS):
        end = pos + sub[i]
        for _ in range(32):
            v, ln = 0, 0
            while (ln, v) not in table or ln == 0:
                v = (v << 1) | ((bits >> pos) & 1)
                pos += 1
                ln += 1
                assert ln <= 16
            s = table[(ln, v)]
            out_sym.append(s)
            if s != 0:
                out_sgn.append((bits >> pos) & 1)
                pos += 1
            else:
                out_sgn.append(None)
        assert pos == end
    x = np.zeros(C)
    kp = [0, 0]
    for j, s in enumerate(out_sym):
        part, a = (0, j) if j < A else (1, j - A)
        if s == 1:
            x[2 * a + part] = -0.0 if out_sgn[j] else 0.0
            continue
        if s == 0:
            u = struct.unpack_from("<Q", b, o)[0]
            o += 8
            kp[part] = ((u & ((1 << 63) - 1)) + (1 << (w - 1))) >> w
            x[2 * a + part] = struct.unpack("<d", struct.pack("<Q", u))[0]
        else:
            kp[part] += s - 2 - 8190
            u = (kp[part] << w) | (out_sgn[j] << 63)
            x[2 * a + part] = struct.unpack("<d", struct.pack("<Q", u))[0]
    assert o == len(b)
    return x


@pytest.mark.parametrize("level", range(1, 6))
def test_independent_decoder_agrees(level):
    rng = np.random.default_rng(40 + level)
    for C in (64, 512):
        for name, x in families(rng, C).items():
            b = oq.encode_pred(x, level)
            ref = oq.decode_chunk(b, C)
            got = py_decode(b, C)
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (name, C)


def test_powers_of_two_closed_form_stream():
    """re a_j = 2^j, im a_j = 0 at level 3 (t = 9): each real part after the
    first is one binade above its predecessor, 2^52 steps of the log
    transform, 2^9 bins: code 512, symbol 2 + 512 + 8190 = 8704; the first
    real part escapes; imaginary parts are zeros (symbol 1).  Counts 1, A-1, A
    give Huffman lengths 2, 2, 1 (the lone leaf of weight A is taken before
    the node of weight A).  Powers of two sit on bin centres: exact."""
    C, A, level = 64, 32, 3
    x = np.zeros(C)
    x[0::2] = 2.0 ** np.arange(A)
    sym, nesc = oq.pred_symbols(x, level)
    assert nesc == 1
    assert list(sym[:A]) == [0] + [8704] * (A - 1) and list(sym[A:]) == [1] * A
    b = oq.encode_pred(x, level)
    cnt = struct.unpack_from("<16H", b, 4)
    assert cnt[0] == 1 and cnt[1] == 2 and sum(cnt) == 3
    assert struct.unpack_from("<3H", b, 36 + 4) == (1, 0, 8704)   # canonical order: (1,sym 1), (2,sym 0), (2,sym 8704)
    # sub-stream bits: re half: escape 2 bits, then 31 x (2 + sign); im half: 32 x (1 + sign)
    assert struct.unpack_from("<2H", b, 36) == (2 + 31 * 3, 32 * 2)
    nbits = 2 + 31 * 3 + 64
    assert len(b) == 36 + 4 + 8 + 4 * ((nbits + 31) // 32) + 8
    y = oq.decode_chunk(b, C)
    assert np.array_equal(y, x)


def heap_cost(counts):
    h = [c for c in counts if c > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def test_huffman_lengths_are_optimal_and_complete():
    rng = np.random.default_rng(9)
    for trial in range(300):
        n = int(rng.integers(1, 300))
        c = np.zeros(16384, dtype=np.uint32)
        idx = rng.choice(16384, size=n, replace=False)
        c[idx] = rng.integers(1, 60, size=n) if trial % 3 else rng.geometric(0.3, size=n)
        ln = oq.pred_huff_lengths(c)
        assert np.all((ln > 0) == (c > 0))
        assert int(np.sum(ln.astype(np.int64) * c)) == heap_cost(c)
        if n > 1:
            assert sum(2.0 ** -int(l) for l in ln[ln > 0]) == 1.0
        assert ln.max() <= 16


def test_fibonacci_counts_stay_within_sixteen_bits():
    """The deepest Huffman tree over C <= 2048 values: Fibonacci counts
    summing to at most 2048 give depth 15 (depth 17 would need 4181)."""
    fib = [1, 1]
    while sum(fib) + fib[-1] + fib[-2] <= 2048:
        fib.append(fib[-1] + fib[-2])
    c = np.zeros(16384, dtype=np.uint32)
    c[:len(fib)] = fib
    ln = oq.pred_huff_lengths(c)
    assert ln.max() == len(fib) - 1 <= 16


def test_malformed_streams_rejected():
    rng = np.random.default_rng(12)
    C = 256
    x = rng.normal(size=C) * 1e-3
    b = bytearray(oq.encode_pred(x, 2))
    bad = []
    bad.append(bytes(b[:-1]))                                       # truncated
    bad.append(bytes(b) + b"\0\0\0\0")                              # trailing bytes
    t = bytearray(b); t[0] |= 0x20; bad.append(bytes(t))             # header bit 5
    t = bytearray(b); struct.pack_into("<H", t, 4, 3); bad.append(bytes(t))   # Kraft sum above 1
    t = bytearray(b); struct.pack_into("<H", t, 36, struct.unpack_from("<H", t, 36)[0] + 1); bad.append(bytes(t))
    t = bytearray(b); t[0] = (t[0] & ~0x1C) | 0; bad.append(bytes(t))  # level 0: no bins
    for k, s in enumerate(bad):
        with pytest.raises(ValueError):
            oq.decode_chunk(s, C)
    with pytest.raises(ValueError):
        oq.encode_pred(x, 0)


def test_prediction_loses_to_solution_c_on_spiky_data_at_tight_bounds():
    """The paper's comparison: on data whose neighbours differ widely (random
    phases, as in QAOA states) the fine bins of 1e-5 catch few codes and
    Solution C keeps the smaller stream; at 1e-1 the bins are wide enough for
    most codes and prediction wins on the same kind of data."""
    rng = np.random.default_rng(13)
    ph = rng.uniform(0, 2 * np.pi, size=1024)
    spiky = np.stack([np.cos(ph), np.sin(ph)], axis=1).reshape(-1) * rng.uniform(0.5, 2, size=2048) * 1e-5
    assert len(oq.encode_pred(spiky, 1)) > len(oq.encode_chunk(spiky, 1))
    assert len(oq.encode_pred(spiky, 5)) < len(oq.encode_chunk(spiky, 5))
    assert math.isfinite(float(np.sum(oq.decode_chunk(oq.encode_pred(spiky, 1), 2048))))
