"""Error paths of the boundary on the GPU: malformed gate records are rejected
before any work (QCZ_E_INVAL, nothing applied, bytes unchanged), and a state
left invalid by a gate that ran out of arena midway in job ranges becomes
usable again by importing a checkpoint image, with a fresh ledger."""
import ctypes

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say

pytestmark = pytest.mark.gpu

QCZ_E_INVAL, QCZ_E_NOMEM, QCZ_E_STATE = -1, -2, -5


def _bad_records(n):
    nan_u1 = cc.h(3).copy()
    nan_u1["m"][0, 5] = np.nan
    inf_diag = cc.t(2).copy()
    inf_diag["m"][0, 2] = np.inf
    tgt_in_ctrl = cc.x(4, controls=(4, 1)).copy()
    big_target = cc.h(0).copy()
    big_target["target"] = n
    big_control = cc.x(1, controls=(0,)).copy()
    big_control["control_mask"] = 1 << n
    same_targets = cc.rzz(2, 2, 0.3).copy()
    empty_mcz = cc.mcz([0, 1]).copy()
    empty_mcz["control_mask"] = 0
    bad_kind = cc.h(0).copy()
    bad_kind["kind"] = 9
    return {"nan matrix entry": nan_u1, "inf phase": inf_diag, "target in control mask": tgt_in_ctrl,
            "target >= n": big_target, "control >= n": big_control, "DIAG2 on one qubit": same_targets,
            "MCZ without controls": empty_mcz, "unknown kind": bad_kind}


def test_malformed_gate_records_apply_nothing():
    from paper_1911_04034_amd import qcz
    n, bl, level = 12, 8, 2
    good = cc.random_circuit_small(n, depth=4, seed=61)
    g = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=64 << 20)
    o = oq.Sim(n, bl, oq.MODE_FIXED, level)
    assert g.apply(good[:20]) == 20 and o.apply(good[:20]) == 20
    before = [g.export_chunk(c) for c in range(g.nchunks)]
    fp0 = g.footprint()
    for name, bad in _bad_records(n).items():
        for pos in (0, 7, 15):   # the bad record first, in the middle, last
            gates = cc.concat([good[20:20 + pos], bad, good[20 + pos:36]])
            say("malformed record (%s) at %d" % (name, pos))
            rc, applied = g.try_apply(gates)
            assert rc == QCZ_E_INVAL and applied == 0, (name, pos, rc, applied)
            assert [g.export_chunk(c) for c in range(g.nchunks)] == before
            fp = g.footprint()
            assert fp["gates_applied"] == fp0["gates_applied"] and fp["compressed_bytes"] == fp0["compressed_bytes"]
    # the state still works and matches the oracle
    assert g.apply(good[20:]) == len(good) - 20 and o.apply(good[20:]) == len(good) - 20
    assert_same_chunks(g, o, "after the rejected records")


def test_import_restores_a_state_left_invalid_by_a_ranged_gate():
    """Qubit n-1 untouched keeps the upper half of the amplitudes zero (half the
    chunks nearly empty); a Hadamard on it then makes every chunk dense and
    the state larger than the arena: its job ranges commit until the arena is
    full and the gate fails midway, leaving the state invalid.  Importing the
    image exported before the gate makes it usable again."""
    from paper_1911_04034_amd import qcz
    n, bl = 14, 8
    low = cc.random_circuit_small(n - 1, depth=8, seed=62)
    o = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    o.apply(low)
    half = o.footprint()["compressed_bytes"]
    peak_low = o.footprint()["max_compressed"]
    full = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    full.apply(cc.concat([low, cc.h(n - 1)]))
    after = full.footprint()["compressed_bytes"]
    cfg = qcz.Config(n, bl, 0, 0, 0, 0, 0, 0, 0)
    pmin = qcz.load().qcz_pool_bytes_min(ctypes.byref(cfg))
    nchunks = 1 << (n - 8)
    arena = (peak_low + after) // 2 + (8 << 10)
    assert peak_low + (16 << 10) < arena < after
    pool = pmin + 2 * (arena - (64 << 10) - 64 * nchunks)
    g = qcz.State(n, bl, mode=qcz.MODE_LOSSLESS, pool_bytes=pool, batch=16, flags=qcz.FLAG_RANGES)
    say("ranged failure: half %d full %d arena %d" % (half, after, arena))
    assert g.apply(low) == len(low)
    assert_same_chunks(g, o, "before the failing gate")
    image, sizes = g.export_state()
    rc, applied = g.try_apply(cc.h(n - 1))
    assert rc == QCZ_E_NOMEM and applied == 0
    rc, applied = g.try_apply(cc.h(0))
    assert rc == QCZ_E_STATE and applied == 0   # the state is invalid until an import
    g.import_state(image, sizes)
    fp = g.footprint()
    assert fp["gates_applied"] == 0 and fp["lossy_steps"] == 0 and fp["fidelity_lower_bound"] == 1.0
    assert fp["level"] == 0 and fp["compressed_bytes"] == half
    assert_same_chunks(g, o, "after the import")
    # a few gates that keep the state's size (permutations and sign flips): a
    # dense 13-qubit state would itself not fit this arena
    more = cc.concat([cc.x(9), cc.x(11), cc.mcz([0, 3, 5]), cc.x(2, controls=(10,)), cc.x(12)])
    assert g.apply(more) == len(more) and o.apply(more) == len(more)
    assert_same_chunks(g, o, "after gates on the imported state")
