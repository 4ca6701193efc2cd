"""Gate-layer fusion: runs of gates whose jobs lie inside single chunks
(in-chunk targets, diagonal gates and multi-controlled Z on any qubits, any
controls) in one decode / encode pass, each chunk taking the gates that touch
it with each gate's truncation applied in registers, leave the oracle's bytes
and ledger (the oracle runs gate by gate)."""
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
    for key in ("gate_launches", "permute_launches"):   # (a run's chunk counts are the run's, per gate)
        assert sg[key] == sp[key], key
    # the fused passes read and write fewer stream bytes than one pass per gate
    assert sg["bytes_read"] < sp["bytes_read"]


@pytest.mark.parametrize("n,bl,level,seed", [(12, 8, 0, 5), (12, 8, 2, 6), (13, 10, 4, 7), (11, 7, 5, 8),
                                              (12, 6, 1, 9), (13, 9, 3, 10)])
def test_fuse_random_gate_mix(n, bl, level, seed):
    """Random gates of every kind: runs form wherever gates with jobs inside
    single chunks follow each other; chunk-pair gates run as before in between."""
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


@pytest.mark.parametrize("level", [0, 2])
def test_fuse_qaoa_layers_gate_by_gate_equal(level):
    """QAOA layers: every Rzz of a layer and the mixers on in-chunk qubits
    form one run; the bytes after each layer are the oracle's."""
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    gates = cc.qaoa(n, 3, 3, 21)[0]
    mode = oq.MODE_LOSSLESS if level == 0 else oq.MODE_FIXED
    g, o = make(n, bl, mode, level, batch=128)
    p = qcz.State(n, bl, mode=mode, level=level, pool_bytes=64 << 20, batch=128)
    say("fused qaoa14 level=%d (%d gates)" % (level, len(gates)))
    for k in range(0, len(gates), 25):
        part = gates[k:k + 25]
        for s_ in (g, o, p):
            s_.apply(part)
        assert_same_chunks(g, o, "after gate %d" % (k + len(part) - 1))
    fg, fo, fp = g.footprint(), o.footprint(), p.footprint()
    assert fg["lossy_steps"] == fo["lossy_steps"] == fp["lossy_steps"]
    assert fg["fidelity_lower_bound"] == fo["fidelity_lower_bound"]
    sg, sp = g.stats(), p.stats()
    assert sg["bytes_read"] < sp["bytes_read"] / 2   # runs of tens of gates per pass


def test_fuse_controls_on_chunk_bits_and_unit_phases():
    """Runs whose gates skip chunks (controls on chunk-index qubits, unit
    phases on a chunk-index qubit, multi-controlled Z): a chunk no gate of the
    run touches keeps its stream, the others take only their gates."""
    import numpy as np
    n, bl, level = 13, 8, 3
    hi = n - 1
    layer = cc.concat([cc.t(hi), cc.cphase(hi, 2, 0.3), cc.x(1, controls=(hi - 1,)), cc.mcz([0, hi - 2, hi]),
                       cc.diag1(hi - 3, 1.0, np.exp(0.4j)), cc.rzz(hi, 3, 0.7), cc.u1(0, np.array([[0, 1], [1, 0]]),
                                                                                      controls=(hi - 1, hi - 4)),
                       cc.diag2(hi - 1, hi, np.exp(1j * np.array([0.0, 0.0, 0.0, 0.9]))), cc.rz(4, 1.1)])
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 30, 11), layer, cc.h(hi - 2), layer,
                       cc.x(hi), cc.h(5), layer])
    g, o = make(n, bl, oq.MODE_FIXED, level, batch=64)
    say("fused runs that skip chunks")
    for k in range(0, len(gates), 16):
        part = gates[k:k + 16]
        assert g.apply(part) == len(part) and o.apply(part) == len(part)
        assert_same_chunks(g, o, "after gate %d" % (k + len(part) - 1))
    assert g.footprint()["lossy_steps"] == o.footprint()["lossy_steps"]


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
