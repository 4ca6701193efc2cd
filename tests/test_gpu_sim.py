"""GPU simulator parity: after every gate the HIP path holds exactly the
oracle's compressed chunks (same bytes), level decisions and footprint."""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say, same_bits

pytestmark = pytest.mark.gpu

MODES = {"lossless": (oq.MODE_LOSSLESS, 0), "fixed": (oq.MODE_FIXED, None), "adaptive": (oq.MODE_ADAPTIVE, 0)}


def make(n, bl, mode, level=0, budget=0, **kw):
    from paper_1911_04034_amd import qcz
    g = qcz.State(n, bl, mode=mode, level=level, budget=budget, pool_bytes=kw.pop("pool_bytes", 64 << 20), **kw)
    o = oq.Sim(n, bl, mode, level, budget)
    return g, o


def test_initial_state_bytes():
    say("create n=12 b=2^8")
    g, o = make(12, 8, oq.MODE_LOSSLESS)
    assert_same_chunks(g, o, "at creation")
    fp = g.footprint()
    assert fp["compressed_bytes"] == o.footprint()["compressed_bytes"]
    assert fp["nchunks"] == 16


@pytest.mark.parametrize("level", [0, 1, 3])
def test_random12_gate_by_gate(level):
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=20, seed=1)
    mode = oq.MODE_LOSSLESS if level == 0 else oq.MODE_FIXED
    g, o = make(n, bl, mode, level)
    for k in range(len(gates)):
        say("rand12 level=%d gate %d kind=%d q=%d" % (level, k, gates[k]["kind"], gates[k]["target"]))
        assert g.apply(gates[k:k + 1]) == 1
        assert o.apply(gates[k:k + 1]) == 1
        assert_same_chunks(g, o, "after gate %d" % k)
    fg, fo = g.footprint(), o.footprint()
    assert fg["compressed_bytes"] == fo["compressed_bytes"]
    assert fg["lossy_steps"] == fo["lossy_steps"]
    assert fg["fidelity_lower_bound"] == pytest.approx(fo["fidelity_lower_bound"], rel=1e-12)
    assert same_bits(g.state(), o.state())


@pytest.mark.parametrize("waves", [2, 4, 8])
@pytest.mark.parametrize("n,bl,level,seed", [(12, 8, 2, 5), (13, 10, 4, 6), (14, 12, 1, 7), (11, 11, 5, 8)])
def test_all_gate_kinds_batched(n, bl, level, seed, waves):
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 120, seed)])
    g, o = make(n, bl, oq.MODE_FIXED, level, batch=16, chunk_waves=waves)
    say("all kinds n=%d bl=%d level=%d waves=%d" % (n, bl, level, waves))
    assert g.apply(gates) == len(gates)
    assert o.apply(gates) == len(gates)
    assert_same_chunks(g, o, "after %d gates" % len(gates))
    assert g.footprint()["compressed_bytes"] == o.footprint()["compressed_bytes"]


def test_adaptive_rule_same_decisions():
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=20, seed=21)
    ref = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    peak = 0
    for k in range(len(gates)):
        ref.apply(gates[k:k + 1])
        peak = max(peak, ref.footprint()["compressed_bytes"])
    budget = int(0.45 * peak)
    g, o = make(n, bl, oq.MODE_ADAPTIVE, 0, budget, batch=32)
    say("adaptive budget=%d" % budget)
    rc_o = o.apply(gates)
    rc_g, applied = g.try_apply(gates)
    fo, fg = o.footprint(), g.footprint()
    if rc_o >= 0:
        assert rc_g == 0 and applied == len(gates)
    else:
        assert rc_g == -2 and applied == -rc_o - 1
    assert fg["level"] == fo["level"] and fg["level"] > 0
    assert fg["compressed_bytes"] == fo["compressed_bytes"] <= budget
    assert fg["lossy_steps"] == fo["lossy_steps"]
    assert_same_chunks(g, o, "after the adaptive run")


def test_out_of_budget_keeps_last_committed_state():
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=10, seed=22)
    probe = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    probe.apply(gates[:5])
    budget = probe.footprint()["compressed_bytes"] + 64
    g, o = make(n, bl, oq.MODE_ADAPTIVE, 0, budget, batch=8)
    rc_o = o.apply(gates)
    rc_g, applied = g.try_apply(gates)
    assert rc_o < 0 and rc_g == -2
    assert applied == -rc_o - 1
    assert_same_chunks(g, o, "after NOMEM")


def test_grover_closed_form_and_graph_replay():
    from paper_1911_04034_amd import qcz
    n, bl, iters = 14, 10, 12
    w = cc.grover_marked(n, 3)
    it = cc.grover_iteration(n, w)
    g, o = make(n, bl, oq.MODE_FIXED, 1, flags=qcz.FLAG_GRAPH, batch=len(it))
    g.apply(cc.grover_prefix(n))
    o.apply(cc.grover_prefix(n))
    for k in range(iters):
        say("grover n=%d iteration %d (graph)" % (n, k))
        g.apply(it)
        o.apply(it)
    assert_same_chunks(g, o, "after grover")
    theta = math.asin(2.0 ** (-n / 2))
    amp = g.read([w])[0]
    assert abs(abs(amp) - abs(math.sin((2 * iters + 1) * theta))) < 1e-3
    s, n2 = g.moments()
    assert abs(n2 - np.sum(np.abs(o.state()) ** 2)) < 1e-12


def test_qft_closed_form():
    n, bl = 12, 8
    x_in = cc.qft_input(n, 2)
    gates = cc.qft(n, x_in)
    g, o = make(n, bl, oq.MODE_FIXED, 1)
    g.apply(gates)
    o.apply(gates)
    assert_same_chunks(g, o, "after qft")
    st = g.state()
    N = 1 << n
    y = np.arange(N)
    rev = np.array([int(format(v, "0%db" % n)[::-1], 2) for v in y])
    ideal = np.exp(2j * np.pi * x_in * rev / N) / math.sqrt(N)
    f_raw = abs(np.vdot(ideal, st))
    assert f_raw >= g.footprint()["fidelity_lower_bound"] - 1e-12
    assert f_raw > 0.999


def test_export_import_roundtrip_and_readout():
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=6, seed=4)
    g, o = make(n, bl, oq.MODE_FIXED, 2)
    g.apply(gates)
    o.apply(gates)
    idx = np.random.default_rng(0).integers(0, 1 << n, size=100)
    assert same_bits(g.read(idx), o.state()[idx])
    # move chunk 3's stream into chunk 7 on both sides
    blob = g.export_chunk(3)
    g.import_chunk(7, blob)
    o.set_chunk(7, blob)
    assert_same_chunks(g, o, "after import")
    assert g.footprint()["compressed_bytes"] == o.footprint()["compressed_bytes"]
    from paper_1911_04034_amd import qcz
    with pytest.raises(qcz.QczError):
        g.import_chunk(1, b"\xff\xff\xff\xff")


def test_compaction_keeps_bytes():
    n, bl = 13, 8
    gates = cc.random_circuit_small(n, depth=20, seed=9)
    from paper_1911_04034_amd import qcz
    pmin = qcz.load().qcz_pool_bytes_min(__import__("ctypes").byref(qcz.Config(n, bl, 1, 3, 0, 0, 0, 0, 0)))
    g, o = make(n, bl, oq.MODE_FIXED, 3, pool_bytes=pmin + (400 << 10))
    say("compaction run pool small")
    assert g.apply(gates) == len(gates)
    o.apply(gates)
    assert g.footprint()["compactions"] > 0
    assert_same_chunks(g, o, "after compactions")


def test_arena_exhausted_keeps_last_committed_state():
    """A pool whose arena cannot hold the lossless state: the gate that
    overflows it stops on the device, is rolled back, compacted for and
    retried once; the call then fails with NOMEM and the state is the
    oracle's after the gates that completed."""
    n, bl = 13, 8
    from paper_1911_04034_amd import qcz
    gates = cc.random_circuit_small(n, depth=12, seed=31)
    pmin = qcz.load().qcz_pool_bytes_min(__import__("ctypes").byref(qcz.Config(n, bl, 0, 0, 0, 0, 0, 0, 0)))
    g, o = make(n, bl, oq.MODE_LOSSLESS, 0, pool_bytes=pmin, batch=16)
    say("arena exhaustion run")
    rc, applied = g.try_apply(gates)
    assert rc == -2 and 0 < applied < len(gates)
    assert g.stats()["stops"] >= 1
    o.apply(gates[:applied])
    assert_same_chunks(g, o, "after arena NOMEM")


def test_autotune_keeps_bytes_and_settles():
    """The launch-shape autotuner only changes how kernels are launched:
    bytes stay the oracle's while it measures and after it has chosen."""
    n, bl = 14, 10
    from paper_1911_04034_amd import qcz
    gates = cc.random_circuit_small(n, depth=40, seed=12)
    g, o = make(n, bl, oq.MODE_FIXED, 2, flags=qcz.FLAG_AUTOTUNE, batch=4)
    assert g.stats()["tuning"] == 1
    say("autotune run")
    for k in range(0, len(gates), 4):
        g.apply(gates[k:k + 4])
        o.apply(gates[k:k + 4])
    st = g.stats()
    assert st["tuning"] == 0
    assert st["chunk_waves"] in (2, 4, 8) and st["grid"] > 0
    assert_same_chunks(g, o, "after autotuning")


@pytest.mark.parametrize("cache", [False, True])
def test_sampled_gates_full_size_grover24(cache):
    """At the benchmark shape (24 qubits, 2^16-amplitude blocks) compare
    sampled gates: the oracle re-runs one unit of the blockwise loop on the
    GPU's exported input chunks and must produce the GPU's output bytes.
    With the block cache most chunks are copies of a leader job's output."""
    n, bl = 24, 16
    from paper_1911_04034_amd import qcz
    w = cc.grover_marked(n, 2)
    it = cc.grover_iteration(n, w)
    g = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=1, pool_bytes=2 << 30, batch=128,
                  flags=qcz.FLAG_CACHE if cache else 0)
    g.apply(cc.grover_prefix(n))
    g.apply(it)
    rng = np.random.default_rng(5)
    cb = g.cb
    for k in range(len(it)):
        gate = it[k:k + 1]
        if k % 9:
            g.apply(gate)
            continue
        touched = [c for c in range(g.nchunks) if oq.chunk_role(gate, cb, c) in (1, 2)]
        sample = touched if len(touched) <= 4 else [int(c) for c in rng.choice(touched, size=4, replace=False)]
        before = {}
        for c in sample:
            before[c] = g.export_chunk(c)
            if oq.chunk_role(gate, cb, c) == 2:
                c1 = c | (1 << (int(gate["target"][0]) - cb))
                before[c1] = g.export_chunk(c1)
        say("grover24 sampled gate %d kind=%d touched=%d" % (k, gate["kind"][0], len(touched)))
        g.apply(gate)
        for c in sample:
            if oq.chunk_role(gate, cb, c) == 1:
                assert g.export_chunk(c) == oq.gate_job(gate, cb, g.C, c, before[c], 1)
            else:
                c1 = c | (1 << (int(gate["target"][0]) - cb))
                r0, r1 = oq.gate_job(gate, cb, g.C, c, before[c], 1, c1, before[c1], 1)
                assert g.export_chunk(c) == r0 and g.export_chunk(c1) == r1
    theta = math.asin(2.0 ** (-n / 2))
    assert abs(abs(g.read([w])[0]) - abs(math.sin(5 * theta))) < 1e-4
    if cache:
        st = g.stats()
        assert st["cache_on"] == 1 and st["cache_hits"] > st["chunks_reencoded"] // 2


def test_sampled_gates_full_size_qft24():
    """QFT-24 at the benchmark shape: controlled phases run as single-chunk
    register gates, Hadamards as in-chunk or paired LDS gates; for sampled
    gates the oracle re-runs one unit of the blockwise loop on the GPU's
    exported input chunks and must produce the GPU's output bytes."""
    n, bl = 24, 16
    from paper_1911_04034_amd import qcz
    gates = cc.qft(n, cc.qft_input(n, 2))
    g = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=1, pool_bytes=2 << 30, batch=128)
    rng = np.random.default_rng(7)
    cb = g.cb
    checked = 0
    for k in range(len(gates)):
        gate = gates[k:k + 1]
        hadamard = int(gate["kind"][0]) == 0 and int(gate["target"][0]) % 5 == 0   # in registers, LDS, paired
        if k % 13 != 5 and not hadamard:
            g.apply(gate)
            continue
        touched = [c for c in range(g.nchunks) if oq.chunk_role(gate, cb, c) in (1, 2)]
        sample = touched if len(touched) <= 4 else [int(c) for c in rng.choice(touched, size=4, replace=False)]
        before = {}
        for c in sample:
            before[c] = g.export_chunk(c)
            if oq.chunk_role(gate, cb, c) == 2:
                c1 = c | (1 << (int(gate["target"][0]) - cb))
                before[c1] = g.export_chunk(c1)
        say("qft24 sampled gate %d kind=%d target=%d touched=%d" % (k, gate["kind"][0], gate["target"][0], len(touched)))
        g.apply(gate)
        for c in sample:
            if oq.chunk_role(gate, cb, c) == 1:
                assert g.export_chunk(c) == oq.gate_job(gate, cb, g.C, c, before[c], 1)
            else:
                c1 = c | (1 << (int(gate["target"][0]) - cb))
                r0, r1 = oq.gate_job(gate, cb, g.C, c, before[c], 1, c1, before[c1], 1)
                assert g.export_chunk(c) == r0 and g.export_chunk(c1) == r1
            checked += 1
    assert checked >= 25


def test_gates_split_into_job_ranges_when_arena_is_short():
    """An arena a sixty-fourth above the largest state holds neither a
    full-state gate's new streams next to the old ones nor, near the peak, a
    sweep into the other arena; such gates run in job ranges with compaction
    between them, and the bytes stay the oracle's."""
    import ctypes
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    gates = cc.random_circuit_small(n, depth=10, seed=41)
    o = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    o.apply(gates)
    peak = o.footprint()["max_compressed"]
    cfg = qcz.Config(n, bl, 0, 0, 0, 0, 0, 0, 0)
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(cfg))
    nchunks = 1 << (n - 8)
    arena = peak + peak // 64 + (16 << 10)
    pool = pmin + 2 * (arena - (64 << 10) - 64 * nchunks)
    g = qcz.State(n, bl, mode=qcz.MODE_LOSSLESS, pool_bytes=pool, batch=16, flags=qcz.FLAG_RANGES)
    say("job ranges: peak %d arena %d" % (peak, arena))
    assert g.apply(gates) == len(gates)
    assert g.stats()["range_gates"] > 0
    assert_same_chunks(g, o, "after ranged gates")
    assert g.footprint()["compressed_bytes"] == o.footprint()["compressed_bytes"]


def test_underestimated_gate_falls_back_to_a_sweep_or_job_ranges():
    """From a state of two-constant chunks one gate makes every chunk dense:
    the planner's estimate is far too low, the whole gate stops on a full
    arena, and the gate then runs as a sweep into the other arena (or in job
    ranges, should the sweep not fit); bytes stay the oracle's."""
    import ctypes
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    gates = cc.concat([cc.grover_prefix(n), cc.random_circuit_small(n, depth=4, seed=43)])
    o = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    o.apply(gates)
    peak = o.footprint()["max_compressed"]
    cfg = qcz.Config(n, bl, 0, 0, 0, 0, 0, 0, 0)
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(cfg))
    nchunks = 1 << (n - 8)
    arena = int(1.5 * peak) + (64 << 10)
    pool = pmin + 2 * (arena - (64 << 10) - 64 * nchunks)
    g = qcz.State(n, bl, mode=qcz.MODE_LOSSLESS, pool_bytes=pool, batch=64, flags=qcz.FLAG_RANGES)
    say("range fallback: peak %d arena %d" % (peak, arena))
    assert g.apply(gates) == len(gates)
    st = g.stats()
    assert st["stops"] >= 1 and st["sweep_gates"] + st["range_gates"] > 0
    assert_same_chunks(g, o, "after the fallback")
