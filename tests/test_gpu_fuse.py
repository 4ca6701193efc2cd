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


def group_heavy(n, seed):
    """Runs of chunk-pair gates on chunk-index qubits (n - 4 .. n - 1 with
    2^10-amplitude chunks): Hadamard and Rx layers, pair gates with controls on
    chunk-index and in-chunk qubits, X with in-chunk controls, between random
    gates of every kind."""
    import numpy as np
    hi = list(range(10, n))
    parts = [cc.concat([cc.h(q) for q in range(n)]), cc.random_unitary_gates(n, 12, seed)]
    for k in range(3):
        parts.append(cc.concat([cc.rx(q, 0.3 + 0.2 * k + 0.01 * q) for q in hi]))
        parts.append(cc.concat([cc.u1(hi[0], np.array([[0, 1j], [1j, 0]]), controls=(hi[1],)),
                                cc.u1(hi[1], np.array([[1, 1], [1, -1]]) / np.sqrt(2), controls=(3,)),
                                cc.x(hi[0], controls=(5,)), cc.h(hi[1]), cc.h(hi[0]),
                                cc.u1(hi[2], np.array([[np.cos(0.4), -np.sin(0.4)], [np.sin(0.4), np.cos(0.4)]]),
                                      controls=(hi[0], 2)), cc.h(hi[3])]))
        parts.append(cc.random_unitary_gates(n, 10, seed + 1 + k))
        parts.append(cc.concat([cc.rzz(hi[0], hi[2], 0.7), cc.rzz(1, hi[3], 0.2)]))
    return cc.concat(parts)


@pytest.mark.parametrize("level", [0, 1, 3])
def test_chunk_group_runs_match_oracle(level):
    """Runs of chunk-pair gates on two chunk-index qubits in one pass over
    groups of four chunks: bytes equal the oracle's (gate by gate) after every
    batch, and to the plain GPU run's."""
    from paper_1911_04034_amd import qcz
    n, bl = 14, 10
    gates = group_heavy(n, 60 + level)
    mode = oq.MODE_LOSSLESS if level == 0 else oq.MODE_FIXED
    g, o = make(n, bl, mode, level, batch=64, flags=qcz.FLAG_FUSE | qcz.FLAG_GROUPS)
    p = qcz.State(n, bl, mode=mode, level=level, pool_bytes=64 << 20, batch=64)
    say("chunk-group runs level=%d (%d gates)" % (level, len(gates)))
    for k in range(0, len(gates), 24):
        part = gates[k:k + 24]
        for s_ in (g, o, p):
            s_.apply(part)
        assert_same_chunks(g, o, "after gate %d" % (k + len(part) - 1))
    fg, fo, fp = g.footprint(), o.footprint(), p.footprint()
    assert fg["lossy_steps"] == fo["lossy_steps"] == fp["lossy_steps"]
    assert fg["fidelity_lower_bound"] == fo["fidelity_lower_bound"]
    assert g.stats()["gate_launches"] == p.stats()["gate_launches"]


def test_chunk_group_runs_qaoa_and_grover_sweeps():
    """QAOA-16 and Grover-15 with fused runs in an arena that a full-state
    gate only fits as a sweep: chunk-group runs also sweep into the other
    arena; bytes equal the oracle's."""
    import ctypes
    from paper_1911_04034_amd import qcz
    for n, gates in ((16, cc.qaoa(16, 2, 3, 17)[0]), (15, cc.grover(15, 2, 19)[0])):
        bl, level = 10, 1
        o = oq.Sim(n, bl, oq.MODE_FIXED, level)
        peak = 0
        for k in range(len(gates)):
            o.apply(gates[k:k + 1])
            peak = max(peak, o.footprint()["compressed_bytes"])
        cfg = qcz.Config(n, bl, 0, 0, 0, qcz.FLAG_FUSE | qcz.FLAG_GROUPS, 0, 0, 0)
        pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(cfg))
        arena = int(1.25 * peak) + (32 << 10)
        pool = pmin + 2 * (arena - (64 << 10) - 64 * (1 << (n - 10)))
        g, o = make(n, bl, oq.MODE_FIXED, level, batch=96, pool_bytes=pool, flags=qcz.FLAG_FUSE | qcz.FLAG_GROUPS)
        say("chunk-group sweeps n=%d: peak %d arena %d" % (n, peak, arena))
        for k in range(0, len(gates), 40):
            part = gates[k:k + 40]
            assert g.apply(part) == len(part) and o.apply(part) == len(part)
            assert_same_chunks(g, o, "n=%d after gate %d" % (n, k + len(part) - 1))
        assert g.stats()["sweep_gates"] > 0


def test_run_that_densifies_the_state_ends_its_batch():
    """Regression: after the Hadamard layer the QAOA state is near-constant,
    and the first layer's run makes it dense.  The chunk-group pass behind it
    in the same call is planned from the sizes the run left, so it sweeps into
    the other arena instead of stopping on a full one (no stop, no
    compaction); bytes equal the oracle's."""
    import ctypes
    from paper_1911_04034_amd import qcz
    n, bl, level = 16, 10, 1
    gates, edges = cc.qaoa(n, 1, 3, 23)
    hadamards = gates[:n]
    layer = gates[n:n + len(edges) + 13]   # Rzz on every edge, Rx on qubits 0 .. 12
    o = oq.Sim(n, bl, oq.MODE_FIXED, level)
    o.apply(hadamards)
    o.apply(layer[:len(edges) + 10])
    dense = o.footprint()["compressed_bytes"]
    cfg = qcz.Config(n, bl, 0, 0, 0, qcz.FLAG_FUSE | qcz.FLAG_GROUPS, 0, 0, 0)
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(cfg))
    arena = int(1.25 * dense) + (32 << 10)
    pool = pmin + 2 * (arena - (64 << 10) - 64 * (1 << (n - 10)))
    g, o = make(n, bl, oq.MODE_FIXED, level, batch=96, pool_bytes=pool, flags=qcz.FLAG_FUSE | qcz.FLAG_GROUPS)
    say("densifying run: dense %d arena %d" % (dense, arena))
    assert g.apply(hadamards) == n and o.apply(hadamards) == n
    assert g.apply(layer) == len(layer) and o.apply(layer) == len(layer)
    assert_same_chunks(g, o, "after the first layer")
    st = g.stats()
    assert st["stops"] == 0 and g.footprint()["compactions"] == 0
    assert st["sweep_gates"] >= 3 and st["kind_bytes"][2] > 0


def test_chunk_group_run_exhausting_the_arena_is_undone():
    """A chunk-group run that overflows the arena stops and is undone over all
    four chunks of every group; the call fails with NOMEM and the state is the
    oracle's after the gates that completed."""
    import ctypes
    from paper_1911_04034_amd import qcz
    n, bl = 14, 10
    gates = cc.concat([cc.h(3), cc.h(7)] + [cc.concat([cc.h(q) for q in range(10, 14)]),
                                            cc.random_unitary_gates(n, 40, 71)])
    flags = qcz.FLAG_FUSE | qcz.FLAG_GROUPS
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(qcz.Config(n, bl, 0, 0, 0, flags, 0, 0, 0)))
    g, o = make(n, bl, oq.MODE_LOSSLESS, 0, pool_bytes=pmin, batch=16, flags=flags)
    rc, applied = g.try_apply(gates)
    say("chunk-group arena exhaustion: rc=%d applied=%d" % (rc, applied))
    assert rc == -2 and 0 < applied < len(gates)
    o.apply(gates[:applied])
    assert_same_chunks(g, o, "after arena NOMEM")


@pytest.mark.parametrize("targets", [(10, 11), (10, 11, 12)])
def test_chunk_group_run_stopped_midway_restores_every_chunk(targets):
    """Regression: a chunk-group run that runs out of arena (as a sweep and
    in place) is rolled back over all chunks of every group (four with two
    target qubits, eight with three), so the call fails with the state
    exactly at the gate before the run.  Two dense chunks (0 and 8 of
    sixteen, in different groups), then Rx on the chunk-index qubits makes
    their groups dense: more than either arena holds."""
    import ctypes
    import math
    import numpy as np
    from paper_1911_04034_amd import qcz
    n, bl = 14, 10
    rot = [cc.u1(q, np.array([[math.cos(0.3 * q + 0.1), -math.sin(0.3 * q + 0.1)],
                              [math.sin(0.3 * q + 0.1), math.cos(0.3 * q + 0.1)]])) for q in range(10)]
    before = cc.concat([cc.h(13)] + rot + [cc.t(q) for q in range(10)])
    run = cc.concat([cc.rx(q, 0.7 + 0.4 * i) for i, q in enumerate(targets)])
    o = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    o.apply(before)
    live = o.footprint()["compressed_bytes"]
    flags = qcz.FLAG_FUSE | qcz.FLAG_GROUPS
    cfg = qcz.Config(n, bl, 0, 0, 0, flags, 0, 0, 0)
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(cfg))
    arena = int(1.8 * live)
    pool = pmin + 2 * (arena - (64 << 10) - 64 * (1 << (n - 10)))
    g = qcz.State(n, bl, mode=qcz.MODE_LOSSLESS, pool_bytes=pool, batch=64, flags=flags)
    assert g.apply(before) == len(before)
    assert_same_chunks(g, o, "before the run")
    say("group run on %s stopped midway: live %d arena %d" % (targets, live, arena))
    rc, applied = g.try_apply(run)
    assert rc == -2 and applied == 0
    assert g.stats()["stops"] >= 1
    assert_same_chunks(g, o, "after the rolled-back run")
    assert g.footprint()["compressed_bytes"] == live


def subnormal_runs(n):
    """Gates that drive some values of a chunk into the subnormal range in
    the middle of a run and bring them back later in the same run: a diagonal
    phase of magnitude 2^-1020 on an in-chunk qubit (every chunk, and with a
    control on a chunk-index qubit only half of them), then its inverse; a
    chunk-pair gate whose first row is scaled by 2^-1020, then a Hadamard on
    the same chunk-index qubit that mixes the small values with normal ones
    (in runs on two chunk-index qubits, then on three).
    Gate by gate, a chunk holding a subnormal value is stored lossless, so a
    run must decide per gate whether to truncate."""
    import numpy as np
    tiny, huge = 2.0 ** -1020, 2.0 ** 1020
    hi = list(range(10, n))
    shrink = np.array([[tiny, tiny], [1.0, -1.0]]) / np.sqrt(2)

    def layer(third):
        # the chunk-pair segment targets two chunk-index qubits, or three
        extra = [cc.rx(hi[2], 0.2)] if third else []
        return cc.concat([cc.rz(0, 0.3), cc.diag1(4, 1.0, tiny), cc.rz(1, 0.5), cc.rx(2, 0.2), cc.rx(5, 0.4),
                          cc.rx(8, 0.25), cc.diag1(4, 1.0, huge), cc.rz(3, 0.1), cc.rx(6, 0.3),
                          cc.diag1(3, 1.0, tiny, controls=(hi[1],)), cc.rx(7, 0.6),
                          cc.diag1(3, 1.0, huge, controls=(hi[1],)),
                          cc.h(hi[0]), cc.h(hi[1]), cc.u1(hi[0], shrink), cc.rx(hi[1], 0.3)] + extra +
                         [cc.h(hi[0]), cc.h(hi[1]), cc.u1(hi[1], shrink, controls=(2,)), cc.h(hi[1]),
                          cc.rx(hi[0], 0.5)])
    return cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 8, 71), layer(False),
                      cc.random_unitary_gates(n, 8, 72), layer(True)])


@pytest.mark.parametrize("level", [1, 3])
@pytest.mark.parametrize("groups", [False, True])
def test_runs_with_subnormal_values_midway(level, groups):
    """Fused runs and chunk-group runs in which values turn subnormal and back
    within the run: the bytes after every batch are the oracle's (which
    re-encodes gate by gate and leaves such chunks untruncated)."""
    from paper_1911_04034_amd import qcz
    n, bl = 13, 10
    gates = subnormal_runs(n)
    flags = qcz.FLAG_FUSE | (qcz.FLAG_GROUPS if groups else 0)
    g, o = make(n, bl, oq.MODE_FIXED, level, batch=64, flags=flags)
    say("runs with subnormal values level=%d groups=%d (%d gates)" % (level, groups, len(gates)))
    for k in range(0, len(gates), 20):
        part = gates[k:k + 20]
        assert g.apply(part) == len(part) and o.apply(part) == len(part)
        assert_same_chunks(g, o, "after gate %d" % (k + len(part) - 1))
    fg, fo = g.footprint(), o.footprint()
    assert fg["lossy_steps"] == fo["lossy_steps"]
    assert fg["compressed_bytes"] == fo["compressed_bytes"]
    if groups:
        assert g.stats()["kind_bytes"][2] > 0   # chunk-group runs formed
