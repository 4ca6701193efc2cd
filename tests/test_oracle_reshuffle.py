"""Oracle pins of Solution D (Sec. 4.2): the real and imaginary parts of a
chunk are separated, then the Solution C steps run on that sequence.  The
stream is the Solution C stream of the separated sequence with header bit 6
set; decoding restores the interleaved order with the same values and error
bound; the reordering helps when the parts lie in different ranges and hurts
when they repeat each other, as the paper's comparison of C and D expects."""
import numpy as np
import pytest

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc

RSH = oq.ENC_RESHUFFLE
DELTA = [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]


def separate(x):
    """re parts first, then im parts (the stored order of Solution D)."""
    return np.concatenate([x[0::2], x[1::2]])


def families(rng, C):
    f = {}
    f["normal"] = rng.normal(size=C)
    f["tiny"] = rng.normal(size=C) * 2.0 ** -40
    s = rng.normal(size=C)
    s[rng.random(C) < 0.7] = 0.0
    f["sparse"] = s
    ph = rng.uniform(0, 2 * np.pi, size=C // 2)
    f["phases"] = np.stack([np.cos(ph), np.sin(ph)], axis=1).reshape(-1) * 2.0 ** -8
    z = np.zeros(C)
    z[::2] = 1.0 + rng.normal(size=C // 2) * 1e-9
    z[1::2] = 2.0 ** -20 * (1.0 + rng.normal(size=C // 2) * 1e-9)
    f["split_ranges"] = z
    few = rng.choice([0.25, -0.25, 0.5], size=C)
    f["few_values"] = few
    return f


@pytest.mark.parametrize("C", [16, 128, 2048])
@pytest.mark.parametrize("level", range(6))
def test_stream_is_solution_c_of_the_separated_parts(C, level):
    rng = np.random.default_rng(10 * C + level)
    for name, x in families(rng, C).items():
        d = oq.encode_chunk(x, level, RSH)
        c = oq.encode_chunk(separate(x), level)
        if c[0] & 3 == 1:        # the separated sequence happens to look like two constants
            continue
        hdr = int.from_bytes(d[:4], "little")
        assert hdr == int.from_bytes(c[:4], "little") | 0x40, name
        assert d[4:] == c[4:], name


@pytest.mark.parametrize("C", [16, 2048])
@pytest.mark.parametrize("level", range(6))
def test_round_trip_values_and_error_bound(C, level):
    rng = np.random.default_rng(70 + C + level)
    for name, x in families(rng, C).items():
        for flags in (RSH, RSH | oq.ENC_ENTROPY):
            y = oq.decode_chunk(oq.encode_chunk(x, level, flags), C)
            ref = oq.decode_chunk(oq.encode_chunk(x, level), C)
            assert np.array_equal(y.view(np.uint64), ref.view(np.uint64)), (name, flags)
            assert np.all(np.abs(y - x) <= DELTA[level] * np.abs(x)), (name, flags)


def test_two_constants_are_never_reshuffled():
    x = np.tile([0.3, -0.7], 64)
    b = oq.encode_chunk(x, 2, RSH)
    assert len(b) == 20 and b[0] & 0x43 == 1
    bad = bytes([b[0] | 0x40]) + b[1:]
    with pytest.raises(ValueError):
        oq.decode_chunk(bad, 128)


def test_unknown_header_bits_rejected():
    rng = np.random.default_rng(3)
    b = oq.encode_chunk(rng.normal(size=128), 1, RSH)
    with pytest.raises(ValueError):
        oq.decode_chunk(bytes([b[0] | 0x80]) + b[1:], 128)


def test_separation_helps_when_parts_lie_in_different_ranges():
    """re near 1, im near 2^-20: interleaved neighbours share no leading byte,
    separated ones share two or more."""
    rng = np.random.default_rng(5)
    x = families(rng, 2048)["split_ranges"]
    for level in range(6):
        assert len(oq.encode_chunk(x, level, RSH)) < len(oq.encode_chunk(x, level)), level


def test_separation_hurts_when_parts_repeat_each_other():
    """re = im for every amplitude: interleaved, every imaginary part repeats
    its neighbour (three leading bytes shared), which separation loses."""
    rng = np.random.default_rng(6)
    a = rng.normal(size=1024)
    x = np.repeat(a, 2)
    for level in range(6):
        assert len(oq.encode_chunk(x, level, RSH)) > len(oq.encode_chunk(x, level)), level


def test_simulator_states_equal_with_and_without_separation():
    """The reordering changes bytes, never values: gate by gate, the states of
    the two codecs agree bit for bit, and every stream re-encoded since
    creation (other than two-constant chunks) carries bit 6."""
    n, bl, level = 11, 7, 2
    gates = cc.concat([cc.random_circuit_small(n, depth=10, seed=7), cc.qft(n, 77)])
    a = oq.Sim(n, bl, oq.MODE_FIXED, level)
    b = oq.Sim(n, bl, oq.MODE_FIXED, level, codec=RSH)
    differ = 0
    for k in range(len(gates)):
        a.apply(gates[k:k + 1])
        b.apply(gates[k:k + 1])
        assert np.array_equal(a.state().view(np.float64), b.state().view(np.float64)), k
        fa, fb = a.footprint(), b.footprint()
        assert fa["lossy_steps"] == fb["lossy_steps"]
        differ += fa["compressed_bytes"] != fb["compressed_bytes"]
    assert differ > 0
    for c in range(b.nchunks):
        h = b.chunk(c)[0]
        assert (h & 3) == 1 or (h & 0x40), c
