"""Pins of the oracle's blockwise compressed simulator (Sec. 3.1, 3.3), its
variable error bound (Sec. 3.7) and fidelity ledger (Sec. 3.8).

* lossless: the compressed simulator must equal the uncompressed one bit for
  bit (truncation is the identity, the codec is exact);
* lossy: after every gate each chunk holds either its old values (the gate
  left it alone) or the truncation of the exact update, and every value the
  gate changed went through the truncation (c.f. Sec. 3.7's range);
* the product bound prod(1 - delta_i) of Eq. (11) is below the measured
  fidelity |<psi_ideal|psi_sim>| of Eq. (9), and reproduces Table 2's Grover
  fidelities;
* the level only rises, and only when the compressed state exceeds the budget.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc

GOLD = os.path.join(os.path.dirname(__file__), "golden")
DELTAS = [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]


def chop(xs, level):
    if level == 0:
        return np.array(xs, dtype=np.float64)
    m = -math.floor(math.log2(DELTAS[level]))
    f, e = np.frexp(np.abs(xs))
    out = np.ldexp(np.floor(np.ldexp(f, m + 1)), e - m - 1)
    return np.copysign(out, xs)


def basis0(n):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    return psi


def bits_equal(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def test_initial_state_is_compressed_basis_state():
    s = oq.Sim(12, 8)
    assert s.chunk(0) == oq.encode_chunk(np.r_[1.0, np.zeros(s.C - 1)], 0)
    for c in range(1, s.nchunks):
        assert s.chunk(c) == oq.encode_chunk(np.zeros(s.C), 0)
    assert bits_equal(s.state(), basis0(12))


@pytest.mark.parametrize("n,bl,seed", [(9, 4, 1), (10, 6, 2), (12, 8, 3), (11, 11, 4), (12, 12, 5)])
def test_lossless_equals_dense_bit_exact(n, bl, seed):
    gates = cc.concat([cc.random_circuit_small(n, depth=6, seed=seed), cc.random_unitary_gates(n, 60, seed)])
    s = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    assert s.apply(gates) == len(gates)
    assert bits_equal(s.state(), oq.apply_dense(basis0(n), n, gates))
    assert s.footprint()["lossy_steps"] == 0


@pytest.mark.parametrize("level", [1, 3, 5])
def test_lossy_step_semantics(level):
    n, bl = 10, 6
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 50, 20 + level)])
    s = oq.Sim(n, bl, oq.MODE_FIXED, level)
    ca = s.C // 2
    prev = s.state()
    for k in range(len(gates)):
        g = gates[k:k + 1]
        exact = oq.apply_dense(prev, n, g)
        assert s.apply(g) == 1
        cur = s.state()
        for c in range(s.nchunks):
            sl = slice(c * ca, (c + 1) * ca)
            old = prev[sl].view(np.float64)
            new = cur[sl].view(np.float64)
            upd = exact[sl].view(np.float64)
            truncated = chop(upd, level)
            if bits_equal(new, old) and not bits_equal(upd, old):
                pytest.fail("gate %d changed chunk %d but it was not rewritten" % (k, c))
            if not bits_equal(new, old):
                assert bits_equal(new, truncated), (k, c)
            else:
                # untouched, or touched with an idempotent result
                assert bits_equal(new, truncated) or bits_equal(upd, old)
            # pointwise relative bound of Sec. 3.7 on what is stored
            nz = upd != 0
            assert np.all(np.abs(new[nz] - upd[nz]) <= DELTAS[level] * np.abs(upd[nz]) + 0.0) or bits_equal(new, old)
        prev = cur


def test_control_on_chunk_bits_leaves_bytes_untouched():
    n, bl = 12, 8                      # chunk = 256 amplitudes: qubits 8..11 index chunks
    s = oq.Sim(n, bl, oq.MODE_FIXED, 2)
    s.apply(cc.concat([cc.h(q) for q in range(n)] + [cc.rz(q, 0.3 + q) for q in range(n)]))
    before = [s.chunk(c) for c in range(s.nchunks)]
    g = cc.u1(3, cc.SQRTX_MAT, controls=(9,))     # control on chunk bit 1
    s.apply(g)
    for c in range(s.nchunks):
        if not (c >> 1) & 1:
            assert s.chunk(c) == before[c]
    assert oq.chunk_role(g, 8, 0) == 0 and oq.chunk_role(g, 8, 2) == 1


def test_x_on_chunk_bit_permutes_bytes():
    n, bl = 12, 8
    s = oq.Sim(n, bl, oq.MODE_FIXED, 1)
    s.apply(cc.random_unitary_gates(n, 30, 8, with_controls=False))
    before = [s.chunk(c) for c in range(s.nchunks)]
    s.apply(cc.x(10))                              # chunk bit 2
    for c in range(s.nchunks):
        assert s.chunk(c) == before[c ^ 4]
    assert s.footprint()["lossy_steps"] == s.footprint()["lossy_steps"]


def test_fidelity_bound_holds_and_ledger_is_product():
    n, bl = 10, 6
    gates = cc.random_circuit_small(n, depth=12, seed=11)
    for level in (1, 3, 5):
        s = oq.Sim(n, bl, oq.MODE_FIXED, level)
        s.apply(gates)
        fp = s.footprint()
        assert fp["fidelity_lower_bound"] == pytest.approx((1 - DELTAS[level]) ** fp["lossy_steps"], rel=1e-12)
        ideal = oq.apply_dense(basis0(n), n, gates)
        sim = s.state()
        f_raw = abs(np.vdot(ideal, sim))                    # Eq. (9)
        assert f_raw >= fp["fidelity_lower_bound"] - 1e-12    # Eq. (11)
        assert f_raw <= 1 + 1e-12
        assert np.linalg.norm(sim) <= 1 + 1e-12                # truncation toward zero


def test_table2_grover_fidelities_are_the_product_bound():
    g = json.load(open(os.path.join(GOLD, "table2_fidelity_bound.json")))
    n, bl = 8, 4
    for row in g["rows"]:
        gates = cc.concat([cc.h(k % n) for k in range(row["gates"])])
        s = oq.Sim(n, bl, oq.MODE_FIXED, 1)
        s.apply(gates)
        fp = s.footprint()
        assert fp["lossy_steps"] == row["gates"]
        assert math.floor(fp["fidelity_lower_bound"] * 1000) / 1000 == row["printed_fidelity"]


def test_adaptive_rule_relaxes_only_when_over_budget():
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=10, seed=21)
    ref = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    sizes = []
    for k in range(len(gates)):
        ref.apply(gates[k:k + 1])
        sizes.append(ref.footprint()["compressed_bytes"])
    budget = int(0.6 * max(sizes))
    s = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    levels = []
    for k in range(len(gates)):
        assert s.apply(gates[k:k + 1]) == 1
        fp = s.footprint()
        levels.append(fp["level"])
        assert fp["compressed_bytes"] <= budget
    assert levels == sorted(levels)
    first = next(k for k, lv in enumerate(levels) if lv > 0)
    # before the first relaxation the run is the lossless run
    assert all(sz <= budget for sz in sizes[:first])
    assert sizes[first] > budget
    # a second run in one call takes the same decisions
    s2 = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    assert s2.apply(gates) == len(gates)
    assert bits_equal(s2.state(), s.state()) and s2.footprint()["level"] == levels[-1]


def test_adaptive_rule_out_of_memory_keeps_last_committed_state():
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=10, seed=22)
    probe = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    probe.apply(gates[:5])
    budget = probe.footprint()["compressed_bytes"] + 64
    s = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    rc = s.apply(gates)
    assert rc < 0
    k = -rc - 1
    assert 5 <= k < len(gates)
    assert s.footprint()["gates_applied"] == k
    t = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    assert t.apply(gates[:k]) == k
    assert bits_equal(t.state(), s.state())


def _replay_smallest_fitting_levels(n, bl, gates, budget):
    """The adaptive rule re-derived from its definition (Sec. 3.7): gate k runs
    at the smallest level >= the previous one whose result fits the budget.
    Each candidate level is tried on a per-block simulator whose blocks all
    hold that level (one uniform level = a fixed-level gate) and undone by
    re-importing the chunks saved before the gate."""
    s = oq.Sim(n, bl, oq.MODE_PERBLOCK, 0)
    nblocks = 1 << (n - bl)
    lev, levels = 0, []
    for k in range(len(gates)):
        saved = [s.chunk(c) for c in range(s.nchunks)]
        while True:
            for b in range(nblocks):
                s.set_block_level(b, lev)
            assert s.apply(gates[k:k + 1]) == 1
            if s.footprint()["compressed_bytes"] <= budget:
                break
            for c, data in enumerate(saved):
                s.set_chunk(c, data)
            lev += 1
            assert lev < oq.N_LEVELS
        levels.append(lev)
    return levels, s


def test_adaptive_rule_takes_the_smallest_fitting_level_at_every_gate():
    # a budget tight enough that some gates must relax more than one level at once
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=12, seed=24)
    ref = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    peak = 0
    for k in range(len(gates)):
        ref.apply(gates[k:k + 1])
        peak = max(peak, ref.footprint()["compressed_bytes"])
    budget = int(0.3 * peak)
    want, replay = _replay_smallest_fitting_levels(n, bl, gates, budget)
    s = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    got = []
    for k in range(len(gates)):
        assert s.apply(gates[k:k + 1]) == 1
        got.append(s.footprint()["level"])
    assert got == want
    assert max(b - a for a, b in zip([0] + want, want)) >= 3   # gates that relaxed by several levels at once
    assert bits_equal(s.state(), replay.state())
    for c in range(s.nchunks):
        assert s.chunk(c) == replay.chunk(c)


def test_footprint_min_max_over_the_run():
    # min / max compressed bytes equal the extremes of the sizes seen after
    # every gate, counting the initial state
    n, bl = 11, 7
    gates = cc.random_circuit_small(n, depth=8, seed=24)
    s = oq.Sim(n, bl, oq.MODE_FIXED, 2)
    trace = [s.footprint()["compressed_bytes"]]
    for k in range(len(gates)):
        s.apply(gates[k:k + 1])
        trace.append(s.footprint()["compressed_bytes"])
    fp = s.footprint()
    assert fp["min_compressed"] == min(trace) and fp["max_compressed"] == max(trace)
    assert min(trace) < trace[0] < max(trace) or min(trace) == trace[0]
    t = oq.Sim(n, bl, oq.MODE_FIXED, 2)
    t.apply(gates)   # one call: the same extremes (tracked after each gate, not per call)
    assert t.footprint()["min_compressed"] == min(trace) and t.footprint()["max_compressed"] == max(trace)
