"""GPU parity of the entropy stage (header bit 5: residual lanes stored raw,
as a constant, or by a canonical Huffman code of at most 8 bits): streams
from the HIP encoder equal the oracle's byte for byte, the HIP decoder
rebuilds the oracle's values (also for streams the oracle was forced to
entropy-code, which exercise every lane mode), and a compressed run with
the stage holds the oracle's chunks after every gate."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say, same_bits
from tests.test_gpu_codec import families

pytestmark = pytest.mark.gpu

C = 2048
ENT = oq.ENC_ENTROPY


def entropy_families(rng):
    fam = families(rng, C)
    mags = rng.normal(size=6) * 2.0 ** -12
    x = mags[rng.integers(0, 6, size=C)] * rng.choice([-1.0, 1.0], size=C)
    x[rng.random(C) < 0.4] = 0.0
    fam["few_values_sparse"] = x
    fam["few_values"] = mags[rng.integers(0, 4, size=C)] * rng.choice([-1.0, 1.0], size=C)
    ph = rng.uniform(0, 2 * np.pi, size=C // 2)
    fam["phases"] = np.stack([np.cos(ph), np.sin(ph)], axis=1).reshape(-1) * 2.0 ** -12
    fam["phases_sparse"] = np.where(rng.random(C) < 0.5, fam["phases"], 0.0)
    skew = rng.normal(size=C) * 2.0 ** -14
    skew[rng.random(C) < 0.8] = 2.0 ** -14
    fam["skewed"] = skew
    return fam


@pytest.mark.parametrize("level", range(6))
def test_entropy_encode_matches_oracle_bytes(level):
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(500 + level)
    fam = entropy_families(rng)
    names = sorted(fam)
    X = np.stack([fam[k] for k in names])
    say("entropy encode level=%d chunks=%d" % (level, len(names)))
    slots, sizes = qcz.encode_chunks(torch.from_numpy(X).cuda(), level, codec_flags=qcz.CODEC_ENTROPY)
    slots, sizes = slots.cpu().numpy(), sizes.cpu().numpy()
    took = 0
    for i, k in enumerate(names):
        ref = oq.encode_chunk(X[i], level, ENT)
        got = slots[i, :sizes[i]].tobytes()
        assert got == ref, (k, level, len(got), len(ref))
        took += (ref[0] >> 5) & 1
    assert took >= 3   # several families take the stage at every level


@pytest.mark.parametrize("level", range(6))
def test_entropy_decode_matches_oracle_values(level):
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(600 + level)
    fam = entropy_families(rng)
    names = sorted(fam)
    streams, refs = [], []
    for k in names:   # the encoder's choice, and the stage forced with every lane mode
        for flags in (ENT, oq.ENC_FORCE_ENT, oq.ENC_FORCE_ENT | oq.ENC_FORCE_CODED):
            b = oq.encode_chunk(fam[k], level, flags)
            if len(b) <= qcz.chunk_cap(C):
                streams.append(b)
                refs.append(oq.decode_chunk(b, C))
    slot = (qcz.chunk_cap(C) + 3) & ~3
    S = np.zeros((len(streams), slot), dtype=np.uint8)
    sz = np.zeros(len(streams), dtype=np.int32)
    for i, b in enumerate(streams):
        S[i, :len(b)] = np.frombuffer(b, dtype=np.uint8)
        sz[i] = len(b)
    say("entropy decode level=%d streams=%d" % (level, len(streams)))
    out = qcz.decode_chunks(torch.from_numpy(S).cuda(), torch.from_numpy(sz).cuda(), C).cpu().numpy()
    for i in range(len(streams)):
        assert same_bits(out[i], refs[i]), (i, level)


def test_entropy_encode_many_chunks():
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(78)
    n = 301
    ph = rng.uniform(0, 2 * np.pi, size=(n, C // 2))
    X = np.stack([np.cos(ph), np.sin(ph)], axis=2).reshape(n, C) * 2.0 ** rng.integers(-30, 0, size=(n, 1))
    X[::5, ::3] = 0.0
    for level in (0, 1, 4):
        say("entropy encode many level=%d" % level)
        slots, sizes = qcz.encode_chunks(torch.from_numpy(X).cuda(), level, codec_flags=qcz.CODEC_ENTROPY)
        slots, sizes = slots.cpu().numpy(), sizes.cpu().numpy()
        for i in range(0, n, 7):
            assert slots[i, :sizes[i]].tobytes() == oq.encode_chunk(X[i], level, ENT), (i, level)
        dec = qcz.decode_chunks(torch.from_numpy(slots).cuda(), torch.from_numpy(sizes).cuda(), C).cpu().numpy()
        assert same_bits(dec, oq.truncate(X, level) if level else X)


def make(n, bl, mode, level=0, budget=0, flags=0, **kw):
    from paper_1911_04034_amd import qcz
    g = qcz.State(n, bl, mode=mode, level=level, budget=budget, pool_bytes=kw.pop("pool_bytes", 64 << 20),
                  flags=flags | qcz.FLAG_ENTROPY, **kw)
    o = oq.Sim(n, bl, mode, level, budget, codec=ENT)
    return g, o


@pytest.mark.parametrize("level", [0, 1, 3, 5])
def test_entropy_simulator_gate_by_gate(level):
    n, bl = 13, 10
    gates = cc.concat([cc.random_circuit_small(n, depth=12, seed=41), cc.qft(n, 1234)])
    mode = oq.MODE_LOSSLESS if level == 0 else oq.MODE_FIXED
    g, o = make(n, bl, mode, level)
    took = 0
    for k in range(len(gates)):
        if k % 25 == 0:
            say("entropy sim level=%d gate %d" % (level, k))
        assert g.apply(gates[k:k + 1]) == 1
        assert o.apply(gates[k:k + 1]) == 1
        assert_same_chunks(g, o, "after gate %d" % k)
        took += sum((o.chunk(c)[0] >> 5) & 1 for c in range(o.nchunks))
    assert took > 0
    fg, fo = g.footprint(), o.footprint()
    assert fg["compressed_bytes"] == fo["compressed_bytes"] and fg["lossy_steps"] == fo["lossy_steps"]
    assert same_bits(g.state(), o.state())


def test_entropy_grover_batched_and_readout():
    from paper_1911_04034_amd import qcz
    n, bl, level = 14, 10, 1
    gates, w = cc.grover(n, 6, 3)
    g, o = make(n, bl, oq.MODE_FIXED, level, batch=64)
    say("entropy grover-14 batched")
    assert g.apply(gates) == len(gates) and o.apply(gates) == len(gates)
    assert_same_chunks(g, o, "after grover-14")
    psi = o.state()
    assert same_bits(g.state(), psi)
    idx = np.array([w, 0, 1, (1 << n) - 1, 777])
    assert same_bits(g.read(idx), psi[idx])
    tot, n2 = g.moments()
    assert abs(n2 - float(np.sum(np.abs(psi) ** 2))) < 1e-12
    plain = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=64 << 20)
    plain.apply(gates)
    ov = g.overlap(plain)   # an entropy state against a state without the stage: the same values
    assert abs(ov - complex(np.vdot(psi, psi))) < 1e-12
    assert g.footprint()["compressed_bytes"] < plain.footprint()["compressed_bytes"]


def test_entropy_adaptive_and_fused_runs():
    from paper_1911_04034_amd import qcz
    n, bl = 13, 10
    gates = cc.concat([cc.grover_prefix(n), cc.random_circuit_small(n, depth=8, seed=42)])
    ref = oq.Sim(n, bl, oq.MODE_LOSSLESS, codec=ENT)
    peak = 0
    for k in range(len(gates)):
        ref.apply(gates[k:k + 1])
        peak = max(peak, ref.footprint()["compressed_bytes"])
    budget = int(0.5 * peak)
    g, o = make(n, bl, oq.MODE_ADAPTIVE, 0, budget, batch=16)
    say("entropy adaptive budget %d" % budget)
    assert g.apply(gates) == len(gates) and o.apply(gates) == len(gates)
    assert_same_chunks(g, o, "after the adaptive run")
    assert g.footprint()["level"] == o.footprint()["level"] > 0
    fused = cc.concat([cc.grover(n, 3, 5)[0]])
    g2, o2 = make(n, bl, oq.MODE_FIXED, 2, flags=qcz.FLAG_FUSE, batch=64)
    say("entropy fused runs")
    assert g2.apply(fused) == len(fused) and o2.apply(fused) == len(fused)
    assert_same_chunks(g2, o2, "after fused runs")


def test_entropy_streams_import_only_where_enabled():
    from paper_1911_04034_amd import qcz
    n, bl = 12, 10
    g, o = make(n, bl, oq.MODE_FIXED, 1)
    gates = cc.random_circuit_small(n, depth=6, seed=43)
    g.apply(gates)
    o.apply(gates)
    c = next(c for c in range(o.nchunks) if (o.chunk(c)[0] >> 5) & 1)
    blob = o.chunk(c)
    plain = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=1, pool_bytes=64 << 20)
    with pytest.raises(qcz.QczError):
        plain.import_chunk(c, blob)
    g2, o2 = make(n, bl, oq.MODE_FIXED, 1)
    g2.import_chunk(c, blob)
    assert g2.export_chunk(c) == blob
    assert same_bits(g2.state()[c * (C // 2):(c + 1) * (C // 2)], o.state()[c * (C // 2):(c + 1) * (C // 2)])
