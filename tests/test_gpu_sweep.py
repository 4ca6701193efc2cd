"""Sweeps: a gate whose new streams do not fit beside the live ones runs as one
launch that writes every chunk into the other arena (the chunks the gate
leaves unchanged, through its controls or unit phases, copied as they are),
and the arenas swap roles.  Bytes, footprint, ledger and level decisions stay
the oracle's after every gate, in every mode."""
import ctypes

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say, same_bits

pytestmark = pytest.mark.gpu


def pool_for(n, bl, arena, flags=0):
    """Pool bytes whose two arenas hold about `arena` bytes each (for a state
    created with `flags`, which may reserve more of the pool)."""
    from paper_1911_04034_amd import qcz
    cfg = qcz.Config(n, bl, 0, 0, 0, flags, 0, 0, 0)
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(cfg))
    nchunks = 1 << (n - min(bl, 10))
    return pmin + 2 * (arena - (64 << 10) - 64 * nchunks)


def peak_of(n, bl, gates, mode=oq.MODE_LOSSLESS, level=0, codec=0):
    o = oq.Sim(n, bl, mode, level, codec=codec)
    peak = 0
    for k in range(len(gates)):
        o.apply(gates[k:k + 1])
        peak = max(peak, o.footprint()["compressed_bytes"])
    return peak


def carry_heavy(n, seed):
    """Gates whose plain enumeration skips chunks (controls on chunk-index
    qubits, diagonal gates with a unit phase on chunk-index qubits), between
    random gates of every kind that keep the state dense."""
    hi = n - 1
    parts = [cc.concat([cc.h(q) for q in range(n)]), cc.random_unitary_gates(n, 24, seed)]
    for k in range(4):
        parts += [cc.x(k, controls=(hi - k,)), cc.t(hi - k), cc.cphase(hi, k + 1, 0.7 + k),
                  cc.mcz([0, hi - 1, hi]), cc.u1(2, np.array([[0, 1j], [1j, 0]]), controls=(hi - 2, hi - 3)),
                  cc.diag1(hi - 1, 1.0, np.exp(0.3j * (k + 1))), cc.rzz(hi, hi - 2, 0.4 + k),
                  cc.h(hi - k, ) if k % 2 else cc.rx(hi - 3, 0.9)]
        parts.append(cc.random_unitary_gates(n, 8, seed + 1 + k))
    return cc.concat(parts)


@pytest.mark.parametrize("level", [0, 2])
def test_sweeps_gate_by_gate(level):
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    gates = carry_heavy(n, 70 + level)
    mode = oq.MODE_LOSSLESS if level == 0 else oq.MODE_FIXED
    peak = peak_of(n, bl, gates, mode, level)
    arena = int(1.2 * peak) + (16 << 10)
    g = qcz.State(n, bl, mode=mode, level=level, pool_bytes=pool_for(n, bl, arena))
    o = oq.Sim(n, bl, mode, level)
    say("sweeps gate by gate: level %d peak %d arena %d" % (level, peak, arena))
    for k in range(len(gates)):
        assert g.apply(gates[k:k + 1]) == 1 and o.apply(gates[k:k + 1]) == 1
        assert_same_chunks(g, o, "after gate %d" % k)
    st, fg, fo = g.stats(), g.footprint(), o.footprint()
    assert st["sweep_gates"] >= 10 and st["range_gates"] == 0
    assert fg["compressed_bytes"] == fo["compressed_bytes"] and fg["lossy_steps"] == fo["lossy_steps"]
    assert fg["fidelity_lower_bound"] == fo["fidelity_lower_bound"]
    assert fg["min_compressed"] == fo["min_compressed"] and fg["max_compressed"] == fo["max_compressed"]
    assert same_bits(g.state(), o.state())


def test_sweeps_in_batches_with_fused_runs():
    from paper_1911_04034_amd import qcz
    n, bl, level = 15, 9, 1
    gates = cc.concat([carry_heavy(n, 80), cc.qft(n, 4321)])
    peak = peak_of(n, bl, gates, oq.MODE_FIXED, level)
    arena = int(1.25 * peak) + (16 << 10)
    for flags in (0, qcz.FLAG_FUSE, qcz.FLAG_FUSE | qcz.FLAG_GRAPH):
        g = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=pool_for(n, bl, arena, flags), flags=flags,
                      batch=32)
        o = oq.Sim(n, bl, oq.MODE_FIXED, level)
        say("sweeps in batches: flags %d peak %d arena %d" % (flags, peak, arena))
        for k in range(0, len(gates), 40):
            part = gates[k:k + 40]
            assert g.apply(part) == len(part) and o.apply(part) == len(part)
            assert_same_chunks(g, o, "after gate %d (flags %d)" % (k + len(part) - 1, flags))
        assert g.stats()["sweep_gates"] > 0
        assert g.footprint()["compressed_bytes"] == o.footprint()["compressed_bytes"]


def test_adaptive_rule_with_sweeps():
    """Sec. 3.7 under a budget of half the lossless peak, in an arena that a
    full-state gate only fits as a sweep: a sweep stopped by the budget is
    undone from the untouched arena and redone one level looser."""
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    gates = carry_heavy(n, 90)
    budget = int(0.5 * peak_of(n, bl, gates))
    arena = int(1.3 * budget) + (16 << 10)
    g = qcz.State(n, bl, mode=qcz.MODE_ADAPTIVE, budget=budget, pool_bytes=pool_for(n, bl, arena))
    o = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    say("adaptive sweeps: budget %d arena %d" % (budget, arena))
    for k in range(len(gates)):
        rg, ro = g.try_apply(gates[k:k + 1]), o.apply(gates[k:k + 1])
        assert rg == (0, 1) and ro == 1, (k, rg, ro)
        assert g.footprint()["level"] == o.footprint()["level"], k
        assert_same_chunks(g, o, "after gate %d" % k)
    st = g.stats()
    assert st["sweep_gates"] > 0 and st["stops"] > 0
    assert g.footprint()["level"] > 0
    assert g.footprint()["fidelity_lower_bound"] == o.footprint()["fidelity_lower_bound"]


def test_entropy_streams_sweep():
    from paper_1911_04034_amd import qcz
    n, bl, level = 15, 10, 1
    gates = cc.concat([cc.grover(n, 2, 7)[0], carry_heavy(n, 95)])
    peak = peak_of(n, bl, gates, oq.MODE_FIXED, level, codec=oq.ENC_ENTROPY)
    arena = int(1.25 * peak) + (32 << 10)
    g = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=pool_for(n, bl, arena, qcz.FLAG_ENTROPY),
                  flags=qcz.FLAG_ENTROPY, batch=16)
    o = oq.Sim(n, bl, oq.MODE_FIXED, level, codec=oq.ENC_ENTROPY)
    say("entropy sweeps: peak %d arena %d" % (peak, arena))
    for k in range(0, len(gates), 16):
        part = gates[k:k + 16]
        assert g.apply(part) == len(part) and o.apply(part) == len(part)
        assert_same_chunks(g, o, "after gate %d" % (k + len(part) - 1))
    assert g.stats()["sweep_gates"] > 0


def test_sweep_without_room_falls_back_and_keeps_the_state():
    """A gate that makes every chunk dense does not fit in the other arena
    either: its sweep stops, is undone, and without job ranges the call fails
    with the state at the last committed gate."""
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    low = cc.random_circuit_small(n - 1, depth=8, seed=62)
    o = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    o.apply(low)
    half, peak_low = o.footprint()["compressed_bytes"], o.footprint()["max_compressed"]
    full = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    full.apply(cc.concat([low, cc.h(n - 1)]))
    after = full.footprint()["compressed_bytes"]
    arena = (peak_low + after) // 2 + (8 << 10)
    assert peak_low + (16 << 10) < arena < after
    g = qcz.State(n, bl, mode=qcz.MODE_LOSSLESS, pool_bytes=pool_for(n, bl, arena), batch=16)
    assert g.apply(low) == len(low)
    rc, applied = g.try_apply(cc.h(n - 1))
    assert rc == -2 and applied == 0
    assert g.stats()["stops"] >= 1
    assert_same_chunks(g, o, "after the failed sweep")
    assert g.footprint()["compressed_bytes"] == half
    more = cc.concat([cc.x(9), cc.mcz([0, 3, 5]), cc.x(2, controls=(10,)), cc.t(12)])
    assert g.apply(more) == len(more) and o.apply(more) == len(more)
    assert_same_chunks(g, o, "after gates on the kept state")
