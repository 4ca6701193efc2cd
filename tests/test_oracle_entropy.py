"""Pins of the oracle's entropy stage (the entropy-coding part of Solution C's
Zstd step, Sec. 4.2, in the project's own chunk format: per-lane canonical
Huffman codes, header bit 5).

* the code construction: Huffman's algorithm is optimal, so on tiny alphabets
  its cost equals the brute-force minimum over all complete prefix codes, and
  equals an independent heap-based Huffman; the Kraft sum is exactly 1 unless
  the 8-bit limit applied, then at most 1; canonical codes are prefix-free and
  ordered; hand-derived examples;
* the byte layout: two hand-derived streams (golden/entropy_chunks.json) and
  a decoder written here from the format text, independently of the C one;
* the codec: decode(encode(x)) equals the truncation of x with the stage on,
  the stage is taken only when strictly smaller, malformed streams are
  rejected;
* the simulator: the entropy stage is lossless, so every decoded state equals
  the run without it, with no more bytes after any gate.
"""
import heapq
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from test_oracle_codec import FAMILIES, chop, chunk_family, same_bits

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ENT = oq.ENC_ENTROPY


# ---------------------------------------------------------------- code lengths
def heap_huffman_cost(counts):
    """Textbook Huffman (merge the two lightest until one tree is left): its
    cost sum(count * depth) equals the sum of the merged weights."""
    h = [c for c in counts if c > 0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def complete_length_vectors(k, maxlen):
    """All length vectors of k symbols whose Kraft sum is exactly 1."""
    for ls in itertools.product(range(1, maxlen + 1), repeat=k):
        if sum(2.0 ** -l for l in ls) == 1.0:
            yield ls


def test_huffman_is_optimal_on_tiny_alphabets_brute_force():
    rng = np.random.default_rng(1)
    for trial in range(150):
        k = int(rng.integers(2, 6))
        nsym = int(rng.integers(k, 17))
        present = rng.choice(nsym, size=k, replace=False)
        counts = np.zeros(nsym, dtype=np.uint32)
        counts[present] = rng.integers(1, 40, size=k)
        lens = oq.huff_lengths(counts)
        assert np.all((lens > 0) == (counts > 0))
        cost = int(np.sum(counts.astype(np.int64) * lens))
        best = min(sum(int(c) * l for c, l in zip(counts[present], ls))
                   for ls in complete_length_vectors(k, k - 1))
        assert cost == best, (counts.tolist(), lens.tolist())


def test_huffman_cost_equals_independent_heap_huffman():
    rng = np.random.default_rng(2)
    for trial in range(400):
        nsym = int(rng.choice([2, 4, 8, 16]))
        counts = rng.integers(0, 200, size=nsym).astype(np.uint32)
        counts[rng.random(nsym) < 0.3] = 0
        if np.count_nonzero(counts) < 2:
            counts[:2] = [3, 5]
        lens = oq.huff_lengths(counts)
        kraft = sum(2.0 ** -int(l) for l in lens if l)
        if lens.max() < 8:   # the limit never acted (a Huffman tree is never deeper than 8 here)
            assert kraft == 1.0
            assert int(np.sum(counts.astype(np.int64) * lens)) == heap_huffman_cost(counts.tolist())
        assert kraft <= 1.0 and lens.max() <= 8


def test_hand_examples_and_ties():
    assert oq.huff_lengths([5, 1, 1, 2]).tolist() == [1, 3, 3, 2]
    assert oq.huff_lengths([1, 1, 1, 1]).tolist() == [2, 2, 2, 2]
    # three equal leaves: the leaf (lowest symbol first) is taken before the
    # equal-weight node, so symbols 0 and 1 join first and symbol 2 stays short
    assert oq.huff_lengths([1, 1, 2]).tolist() == [2, 2, 1]
    assert oq.huff_lengths([2, 1, 1]).tolist() == [1, 2, 2]
    assert oq.huff_lengths([0, 7, 0, 7]).tolist() == [0, 1, 0, 1]
    with pytest.raises(ValueError):
        oq.huff_lengths([0, 9, 0])


def test_length_limit_on_fibonacci_counts():
    fib = [1, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 377, 610, 987]
    # an unlimited Huffman tree of these weights is a path of depth 15
    lens = oq.huff_lengths(fib)
    assert lens.max() == 8
    units = sum(1 << (8 - int(l)) for l in lens)
    assert units <= 256
    assert oq.huff_lengths(fib[:12]).tolist() == [8, 8, 8, 8, 8, 8, 7, 5, 4, 3, 2, 1]


def test_canonical_codes():
    # lengths 2, 1, 3, 3 -> symbol 1 gets 0, symbol 0 gets 10, then 110, 111
    assert oq.canon_codes([2, 1, 3, 3]).tolist() == [0b10, 0b0, 0b110, 0b111]
    rng = np.random.default_rng(3)
    for trial in range(100):
        counts = rng.integers(0, 50, size=16).astype(np.uint32)
        counts[:2] = [1, 2]
        lens = oq.huff_lengths(counts)
        codes = oq.canon_codes(lens)
        words = [format(int(codes[s]), "0%db" % lens[s]) for s in range(16) if lens[s]]
        for a, b in itertools.permutations(words, 2):
            assert not b.startswith(a)
        order = sorted((int(lens[s]), s) for s in range(16) if lens[s])
        vals = [int(codes[s]) << (8 - int(lens[s])) for _, s in order]
        assert vals == sorted(vals) and len(set(vals)) == len(vals)


# ---------------------------------------------------------------- byte layout
def test_golden_entropy_chunks():
    g = json.load(open(os.path.join(GOLD, "entropy_chunks.json")))
    x = np.array(g["values"])
    a = oq.encode_chunk(x, g["level"], oq.ENC_FORCE_ENT)
    b = oq.encode_chunk(x, g["level"], oq.ENC_FORCE_ENT | oq.ENC_FORCE_CODED)
    assert a.hex() == g["chunks"]["a_forced_entropy"]
    assert b.hex() == g["chunks"]["b_forced_coded_lanes"]
    for blob in (a, b):
        assert same_bits(oq.decode_chunk(blob, x.size), chop(x, g["level"]))
        assert same_bits(py_decode(blob, x.size), chop(x, g["level"]))


class Bits:
    def __init__(self, data, pos=0):
        self.data, self.pos = data, pos

    def get(self, n):
        v = 0
        for k in range(n):
            p = self.pos + k
            v |= ((self.data[p >> 3] >> (p & 7)) & 1) << k
        self.pos += n
        return v


SIG = [64, 29, 26, 22, 19, 16]


def py_decode(blob, C):
    """The format text, decoded in plain Python (PACK / SPARSE / CONST2, with
    or without the entropy stage); returns float64 values."""
    hdr = int.from_bytes(blob[:4], "little")
    mode, lev, ent = hdr & 3, (hdr >> 2) & 7, (hdr >> 5) & 1
    K = SIG[lev]
    if mode == 1:
        t = [int.from_bytes(blob[4:12], "little"), int.from_bytes(blob[12:20], "little")]
        return np.array([t[i & 1] for i in range(C)], dtype=np.uint64).view(np.float64)
    off = 4
    if mode == 2:
        bm = Bits(blob, 8 * off)
        pos = [i for i in range(C) if bm.get(1)]
        off += 4 * ((C + 31) // 32)
    else:
        pos = list(range(C))
    N = len(pos)
    cb = Bits(blob, 8 * off)
    L = [cb.get(2) for _ in range(N)]
    off += 4 * ((N + 15) // 16)
    vals = []
    prev = 0
    top = lambda nb: 0 if nb == 0 else ((1 << 64) - 1) ^ ((1 << (64 - nb)) - 1)
    if not ent:
        rb = Bits(blob, 8 * off)
        for i in range(N):
            r = max(0, K - 8 * L[i])
            R = rb.get(r)
            v = (prev & top(8 * L[i])) | (R if K >= 64 else R << (64 - K))
            vals.append(v)
            prev = v
    else:
        NN = (K + 3) // 4
        width = [min(4, K - 4 * j) for j in range(NN)]
        word = int.from_bytes(blob[off:off + 4], "little")
        modes = [(word >> (2 * j)) & 3 for j in range(NN)]
        assert word >> (2 * NN) == 0 and all(m < 3 for m in modes)
        off += 4
        tb = Bits(blob, 8 * off)
        const, codebook = {}, {}
        for j in range(NN):
            if modes[j] == 1:
                const[j] = tb.get(4)
            elif modes[j] == 2:
                lens = [tb.get(4) for _ in range(1 << width[j])]
                code, prevl, book = -1, 0, {}
                for l, s in sorted((l, s) for s, l in enumerate(lens) if l):
                    code = 0 if code < 0 else (code + 1) << (l - prevl)
                    prevl = l
                    book[(l, code)] = s
                codebook[j] = book
        ntab = sum(1 if m == 1 else (1 << width[j]) if m == 2 else 0 for j, m in enumerate(modes))
        off += 4 * ((ntab + 7) // 8)
        nsub = (C + 15) // 16
        sl = Bits(blob, 8 * off)
        sub_len = [sl.get(12) for _ in range(nsub)]
        off += 4 * ((12 * nsub + 31) // 32)
        bs = Bits(blob, 8 * off)
        i = 0
        for s in range(nsub):
            start = bs.pos
            while i < N and pos[i] < 16 * (s + 1):
                v = prev & top(8 * L[i])
                for j in range(2 * L[i], NN):
                    if modes[j] == 0:
                        sym = bs.get(width[j])
                    elif modes[j] == 1:
                        sym = const[j]
                    else:
                        acc, l = 0, 0
                        while (l, acc) not in codebook[j] or l == 0:
                            acc = (acc << 1) | bs.get(1)
                            l += 1
                            if (l, acc) in codebook[j]:
                                break
                        sym = codebook[j][(l, acc)]
                    v |= sym << (64 - 4 * j - width[j])
                vals.append(v)
                prev = v
                i += 1
            assert bs.pos - start == sub_len[s]
    out = np.zeros(C, dtype=np.uint64)
    out[pos] = np.array(vals, dtype=np.uint64)
    return out.view(np.float64)


def grover_like(rng, C):
    """Few distinct values with sign patterns and zeros (the least
    compressible Grover states hold a handful of magnitudes)."""
    mags = rng.normal(size=6) * 2.0 ** -12
    x = mags[rng.integers(0, 6, size=C)] * rng.choice([-1.0, 1.0], size=C)
    x[rng.random(C) < 0.4] = 0.0
    return x


def qft_like(rng, C):
    ph = rng.uniform(0, 2 * np.pi, size=C // 2)
    return np.stack([np.cos(ph), np.sin(ph)], axis=1).reshape(-1) * 2.0 ** -12


@pytest.mark.parametrize("C", [16, 128, 2048])
@pytest.mark.parametrize("level", range(6))
def test_roundtrip_with_entropy_stage(C, level):
    rng = np.random.default_rng(100 * C + level)
    took = 0
    for kind in FAMILIES + ["grover_like", "qft_like"]:
        x = grover_like(rng, C) if kind == "grover_like" else qft_like(rng, C) if kind == "qft_like" \
            else chunk_family(rng, C, kind)
        plain = oq.encode_chunk(x, level)
        blob = oq.encode_chunk(x, level, ENT)
        assert len(blob) <= len(plain) <= oq.chunk_cap(C)
        hdr = int.from_bytes(blob[:4], "little")
        if hdr & 0x20:
            took += 1
            assert len(blob) < len(plain)
            assert hdr & 3 == int.from_bytes(plain[:4], "little") & 3   # the same body, entropy-coded
        else:
            assert blob == plain
        want = chop(x, level)
        assert same_bits(oq.decode_chunk(blob, C), want), (kind, C, level)
        assert same_bits(py_decode(blob, C), want), (kind, C, level)
        forced = oq.encode_chunk(x, level, oq.ENC_FORCE_ENT)
        for f in (forced, oq.encode_chunk(x, level, oq.ENC_FORCE_ENT | oq.ENC_FORCE_CODED)):
            assert same_bits(oq.decode_chunk(f, C), want) and same_bits(py_decode(f, C), want)
    if C == 2048:
        assert took >= 2   # the dense families take the stage at full chunk size


def test_entropy_stage_gains_on_dense_and_few_value_chunks():
    rng = np.random.default_rng(5)
    for maker, level, gain in ((qft_like, 1, 1.15), (grover_like, 1, 1.3)):
        x = maker(rng, 2048)
        assert len(oq.encode_chunk(x, level)) > gain * len(oq.encode_chunk(x, level, ENT))


def test_malformed_entropy_streams_are_rejected():
    rng = np.random.default_rng(6)
    x = qft_like(rng, 128)
    blob = bytearray(oq.encode_chunk(x, 2, oq.ENC_FORCE_ENT | oq.ENC_FORCE_CODED))
    codes = 4 * (128 // 16)
    lw = 4 + codes
    word = int.from_bytes(blob[lw:lw + 4], "little")
    bad = bytearray(blob)
    bad[lw:lw + 4] = (word | (3 << 2)).to_bytes(4, "little")         # lane mode 3
    with pytest.raises(ValueError):
        oq.decode_chunk(bytes(bad), 128)
    bad = bytearray(blob)
    bad[lw:lw + 4] = (word | (1 << 30)).to_bytes(4, "little")        # a lane past NN
    with pytest.raises(ValueError):
        oq.decode_chunk(bytes(bad), 128)
    for cut in (1, 5, len(blob) // 2):                                # truncated
        with pytest.raises(ValueError):
            oq.decode_chunk(bytes(blob[:-cut]), 128)
    with pytest.raises(ValueError):                                   # trailing byte
        oq.decode_chunk(bytes(blob) + b"\0", 128)
    c2 = bytearray(oq.encode_chunk(np.tile([0.5, 0.25], 64), 1))
    c2[0] |= 0x20                                                     # E on a CONST2 chunk
    with pytest.raises(ValueError):
        oq.decode_chunk(bytes(c2), 128)
    first_coded = next(j for j in range(8) if (word >> (2 * j)) & 3 == 2)
    tb = lw + 4
    nib = sum(1 if (word >> (2 * j)) & 3 == 1 else 16 if (word >> (2 * j)) & 3 == 2 else 0 for j in range(first_coded))
    bad = bytearray(blob)
    for k in range(16):                                               # Kraft sum 16 * 2^-1 > 1
        p = nib + k
        bad[tb + p // 2] = (bad[tb + p // 2] & (0xF0 if p % 2 == 0 else 0x0F)) | (1 << (4 * (p % 2)))
    with pytest.raises(ValueError):
        oq.decode_chunk(bytes(bad), 128)
    assert same_bits(oq.decode_chunk(bytes(blob), 128), chop(x, 2))


@pytest.mark.parametrize("level", [0, 1, 3])
def test_simulator_entropy_stage_is_lossless(level):
    n, bl = 12, 10
    gates = cc.concat([cc.random_circuit_small(n, depth=10, seed=31), cc.qft(n, 77)])
    mode = oq.MODE_LOSSLESS if level == 0 else oq.MODE_FIXED
    a = oq.Sim(n, bl, mode, level)
    b = oq.Sim(n, bl, mode, level, codec=ENT)
    took = 0
    for k in range(len(gates)):
        a.apply(gates[k:k + 1])
        b.apply(gates[k:k + 1])
        assert same_bits(a.state().view(np.float64), b.state().view(np.float64))
        assert b.footprint()["compressed_bytes"] <= a.footprint()["compressed_bytes"]
        took += any(b.chunk(c)[0] & 0x20 for c in range(b.nchunks))
    fa, fb = a.footprint(), b.footprint()
    assert fa["fidelity_lower_bound"] == fb["fidelity_lower_bound"] and fa["lossy_steps"] == fb["lossy_steps"]
    assert took > 0 and fb["compressed_bytes"] < fa["compressed_bytes"]
