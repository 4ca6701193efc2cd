"""Compressed block cache (Sec. 3.4) on the GPU: a job whose input streams
and gate action equal another job's copies that job's output.  The cache
changes no byte: after every circuit the chunks are the oracle's, which
knows nothing of the cache."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say

pytestmark = pytest.mark.gpu


def make(n, bl, mode, level=0, budget=0, flags=None, **kw):
    from paper_1911_04034_amd import qcz
    if flags is None:
        flags = qcz.FLAG_CACHE
    g = qcz.State(n, bl, mode=mode, level=level, budget=budget, pool_bytes=64 << 20, flags=flags, **kw)
    o = oq.Sim(n, bl, mode, level, budget)
    return g, o


@pytest.mark.parametrize("collide", [False, True])
@pytest.mark.parametrize("n,bl,level,seed", [(12, 8, 2, 5), (13, 10, 4, 6), (14, 8, 1, 7), (11, 7, 5, 8)])
def test_cache_all_gate_kinds(n, bl, level, seed, collide):
    """Every gate kind (in-chunk, paired chunks, controls and diagonal
    targets on chunk-index bits) from a state with many equal chunks; with
    `collide` the keys keep 3 bits, so unequal streams share keys and only
    the byte comparison keeps them apart."""
    from paper_1911_04034_amd import qcz
    flags = qcz.FLAG_CACHE | (qcz.FLAG_CACHE_COLLIDE if collide else 0)
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 120, seed)])
    g, o = make(n, bl, oq.MODE_FIXED, level, flags=flags, batch=16)
    say("cache all kinds n=%d bl=%d level=%d collide=%s" % (n, bl, level, collide))
    assert g.apply(gates) == len(gates)
    assert o.apply(gates) == len(gates)
    assert_same_chunks(g, o, "after %d gates" % len(gates))
    assert g.footprint()["compressed_bytes"] == o.footprint()["compressed_bytes"]
    st = g.stats()
    assert st["cache_gates"] > 0 and st["cache_hits"] > 0


def test_cache_grover_gate_by_gate():
    n, bl, level = 14, 8, 1
    w = cc.grover_marked(n, 3)
    it = cc.grover_iteration(n, w)
    g, o = make(n, bl, oq.MODE_FIXED, level)
    g.apply(cc.grover_prefix(n))
    o.apply(cc.grover_prefix(n))
    for r in range(2):
        for k in range(len(it)):
            say("cache grover14 iteration %d gate %d" % (r, k))
            g.apply(it[k:k + 1])
            o.apply(it[k:k + 1])
            assert_same_chunks(g, o, "after iteration %d gate %d" % (r, k))
    st = g.stats()
    # Grover's unmarked chunks repeat: most re-encoded chunks are copies
    assert st["cache_on"] == 1 and st["cache_hits"] > st["chunks_reencoded"] // 2


def test_cache_adaptive_redo_same_decisions():
    """Budget overflows stop a cached gate on the device; its undo log is
    written by both job launches, so the rollback and the redo at the next
    level end where the oracle ends."""
    n, bl = 12, 8
    gates = cc.concat([cc.grover_prefix(n), cc.random_circuit_small(n, depth=20, seed=21)])
    ref = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    peak = 0
    for k in range(len(gates)):
        ref.apply(gates[k:k + 1])
        peak = max(peak, ref.footprint()["compressed_bytes"])
    budget = int(0.45 * peak)
    g, o = make(n, bl, oq.MODE_ADAPTIVE, 0, budget, batch=32)
    say("cache adaptive budget=%d" % budget)
    rc_o = o.apply(gates)
    rc_g, applied = g.try_apply(gates)
    if rc_o >= 0:
        assert rc_g == 0 and applied == len(gates)
    else:
        assert rc_g == -2 and applied == -rc_o - 1
    fo, fg = o.footprint(), g.footprint()
    assert fg["level"] == fo["level"] and fg["level"] > 0
    assert fg["compressed_bytes"] == fo["compressed_bytes"]
    assert g.stats()["stops"] >= 1
    assert_same_chunks(g, o, "after the adaptive run")


def test_cache_switches_off_after_misses():
    """Sec. 3.4: the cache is disabled when it keeps missing.  The rule
    (32 cached gates in a row without a hit) is replayed from the per-gate
    hit counts and must agree with the library's switch."""
    n, bl, level = 12, 8, 3
    gates = cc.random_circuit_small(n, depth=40, seed=3)
    g, o = make(n, bl, oq.MODE_FIXED, level)
    run, on, switched = 0, True, None
    for k in range(len(gates)):
        before = g.stats()
        g.apply(gates[k:k + 1])
        after = g.stats()
        ran = after["cache_gates"] - before["cache_gates"]
        hits = after["cache_hits"] - before["cache_hits"]
        if ran:
            assert on
            run = 0 if hits else run + 1
            if run >= 32:
                on, switched = False, k
        assert after["cache_on"] == (1 if on else 0), "gate %d" % k
    say("cache switched off after gate %s" % switched)
    assert switched is not None
    o.apply(gates)
    assert_same_chunks(g, o, "after the run")


def test_cache_rejected_with_autotune():
    from paper_1911_04034_amd import qcz
    with pytest.raises(qcz.QczError):
        qcz.State(10, 8, mode=qcz.MODE_FIXED, level=1, pool_bytes=16 << 20,
                  flags=qcz.FLAG_CACHE | qcz.FLAG_AUTOTUNE)


def test_cache_flag_with_one_job_per_gate():
    """Two chunks (one job per gate): nothing to share, no gate goes through
    the cache and the bytes are the oracle's."""
    n, bl, level = 11, 11, 5
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 60, 8)])
    g, o = make(n, bl, oq.MODE_FIXED, level, batch=16)
    assert g.apply(gates) == len(gates)
    o.apply(gates)
    assert_same_chunks(g, o, "after %d gates" % len(gates))
    assert g.stats()["cache_gates"] == 0


def test_cache_with_graph_replay():
    """Cached gates captured in HIP graphs (planning, leaders, copies, other
    followers: kernels only, no memset nodes) and replayed: every replay of
    the Grover iteration leaves the oracle's bytes, with eager readouts and
    synchronisations between the replays."""
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    w = cc.grover_marked(n, 5)
    it = cc.grover_iteration(n, w)
    g, o = make(n, bl, oq.MODE_FIXED, 1, flags=qcz.FLAG_CACHE | qcz.FLAG_GRAPH, batch=len(it))
    g.apply(cc.grover_prefix(n))
    o.apply(cc.grover_prefix(n))
    for k in range(4):
        say("cache + graph grover14 iteration %d" % k)
        g.apply(it)
        o.apply(it)
        assert_same_chunks(g, o, "after replay %d" % k)
        assert abs(g.read([w])[0]) > 0.0
    assert g.stats()["cache_hits"] > 0
