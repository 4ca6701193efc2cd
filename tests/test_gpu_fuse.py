"""Gate-layer fusion: runs of in-chunk single-qubit gates in one decode /
encode pass, with each gate's truncation applied in registers, leave the
oracle's bytes and ledger (the oracle runs gate by gate)."""
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say

pytestmark = pytest.mark.gpu


def make(n, bl, mode, level, **kw):
    from paper_1911_04034_amd import qcz
    g = qcz.State(n, bl, mode=mode, level=level, pool_bytes=kw.pop("pool_bytes", 64 << 20),
                  flags=kw.pop("flags", qcz.FLAG_FUSE), **kw)
    return g, oq.Sim(n, bl, mode, level, 0)


def test_fuse_grover_iterations_match_oracle_and_plain_run():
    from paper_1911_04034_amd import qcz
    n, bl, level = 14, 8, 1
    w = cc.grover_marked(n, 3)
    it = cc.grover_iteration(n, w)
    g, o = make(n, bl, oq.MODE_FIXED, level, batch=len(it))
    p = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=64 << 20, batch=len(it))
    for s in (g, o, p):
        s.apply(cc.grover_prefix(n))
    for k in range(4):
        say("fused grover14 iteration %d" % k)
        for s in (g, o, p):
            s.apply(it)
        assert_same_chunks(g, o, "after iteration %d" % k)
    fg, fo, fp = g.footprint(), o.footprint(), p.footprint()
    assert fg["compressed_bytes"] == fo["compressed_bytes"]
    assert fg["lossy_steps"] == fo["lossy_steps"] == fp["lossy_steps"]
    assert fg["fidelity_lower_bound"] == fp["fidelity_lower_bound"]
    sg, sp = g.stats(), p.stats()
    for key in ("gate_launches", "chunks_reencoded", "amps_touched", "permute_launches"):
        assert sg[key] == sp[key], key
    # the fused passes read and write fewer stream bytes than one pass per gate
    assert sg["bytes_read"] < sp["bytes_read"]


@pytest.mark.parametrize("n,bl,level,seed", [(12, 8, 0, 5), (12, 8, 2, 6), (13, 10, 4, 7), (11, 7, 5, 8)])
def test_fuse_random_gate_mix(n, bl, level, seed):
    """Random gates of every kind: runs form wherever in-chunk single-qubit
    gates follow each other; all other gates run as before in between."""
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 150, seed)])
    mode = oq.MODE_LOSSLESS if level == 0 else oq.MODE_FIXED
    g, o = make(n, bl, mode, level, batch=32)
    say("fused random mix n=%d bl=%d level=%d" % (n, bl, level))
    assert g.apply(gates) == len(gates)
    o.apply(gates)
    assert_same_chunks(g, o, "after %d gates" % len(gates))
    fg, fo = g.footprint(), o.footprint()
    assert fg["compressed_bytes"] == fo["compressed_bytes"]
    assert fg["lossy_steps"] == fo["lossy_steps"]
    assert fg["fidelity_lower_bound"] == pytest.approx(fo["fidelity_lower_bound"], rel=1e-12)


def test_fuse_arena_exhausted_keeps_last_committed_state():
    """A fused run that overflows the arena stops on the device and is undone
    as a whole; after compaction and the retry the call fails with NOMEM and
    the state is the oracle's after the gates that completed."""
    import ctypes
    from paper_1911_04034_amd import qcz
    n, bl = 13, 8
    gates = cc.random_circuit_small(n, depth=12, seed=31)
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(qcz.Config(n, bl, 0, 0, 0, qcz.FLAG_FUSE, 0, 0, 0)))
    g, o = make(n, bl, oq.MODE_LOSSLESS, 0, pool_bytes=pmin, batch=16)
    rc, applied = g.try_apply(gates)
    say("fused arena exhaustion: rc=%d applied=%d" % (rc, applied))
    assert rc == -2 and 0 < applied < len(gates)
    o.apply(gates[:applied])
    assert_same_chunks(g, o, "after arena NOMEM")


def test_fuse_rejected_with_autotune():
    from paper_1911_04034_amd import qcz
    with pytest.raises(qcz.QczError):
        qcz.State(10, 8, mode=qcz.MODE_FIXED, level=1, pool_bytes=16 << 20, flags=qcz.FLAG_FUSE | qcz.FLAG_AUTOTUNE)
