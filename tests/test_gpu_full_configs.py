"""Full-size configuration: the 30-qubit 5x6-grid random circuit of depth 20
with 2^20-amplitude blocks at bound 1e-4 (16 GiB uncompressed).  Sampled
gates are re-run by the oracle on the GPU's exported input chunks (one unit
of the blockwise loop each) and must give the GPU's output bytes; the end
state's fidelity against the uncompressed fp64 run is measured (Eq. (9))."""
import math

import numpy as np
import pytest

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def sampled_check(g, gate, level, rng, tries=64, want=3):
    """Export a few chunks the gate touches, apply it, compare with the oracle."""
    cb = g.cb
    picks = []
    for c in rng.integers(0, g.nchunks, size=tries):
        c = int(c)
        role = oq.chunk_role(gate, cb, c)
        if role == 3:                                    # high half of a pair: use the low one
            c &= ~(1 << (int(gate["target"][0]) - cb))
            role = 2
        if role in (1, 2) and c not in picks:
            picks.append(c)
        if len(picks) == want:
            break
    before = {}
    for c in picks:
        before[c] = g.export_chunk(c)
        if oq.chunk_role(gate, cb, c) == 2:
            c1 = c | (1 << (int(gate["target"][0]) - cb))
            before[c1] = g.export_chunk(c1)
    g.apply(gate)
    for c in picks:
        if oq.chunk_role(gate, cb, c) == 1:
            assert g.export_chunk(c) == oq.gate_job(gate, cb, g.C, c, before[c], level)
        else:
            c1 = c | (1 << (int(gate["target"][0]) - cb))
            r0, r1 = oq.gate_job(gate, cb, g.C, c, before[c], level, c1, before[c1], level)
            assert g.export_chunk(c) == r0 and g.export_chunk(c1) == r1
    return len(picks)


def test_grid30_full_size_sampled_gates_and_fidelity():
    import torch
    from paper_1911_04034_amd import qcz
    import dense_ref as ref
    n, bl, level = 30, 20, 2
    gates = cc.grid_rcs(5, 6, 20, 3)
    g = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=level, pool_bytes=40 << 30, batch=128)
    rng = np.random.default_rng(30)
    checked = 0
    k = 0
    marks = set(int(x) for x in np.linspace(0, len(gates) - 1, 12))
    while k < len(gates):
        nxt = min([m for m in marks if m >= k] + [len(gates)])
        if nxt > k:
            g.apply(gates[k:nxt])
            k = nxt
            continue
        say("grid30 sampled gate %d kind=%d target=%d" % (k, gates[k]["kind"], gates[k]["target"]))
        checked += sampled_check(g, gates[k:k + 1], level, rng)
        k += 1
    assert checked >= 20
    fp = g.footprint()
    say("grid30 compressed %.2f GB ratio %.3f min ratio %.3f F_lb %.6f" % (
        fp["compressed_bytes"] / 1e9, fp["ratio"], fp["raw_bytes"] / (fp["max_compressed"] + fp["table_bytes"]),
        fp["fidelity_lower_bound"]))
    psi = ref.run(gates, n)
    ov, n2 = ref.overlap_with_compressed(psi, g)
    f_raw, f_norm = abs(ov), abs(ov) / math.sqrt(n2)
    say("grid30 fidelity raw %.6f norm %.6f" % (f_raw, f_norm))
    assert f_norm >= 0.99 and f_raw >= fp["fidelity_lower_bound"]
    del psi
    torch.cuda.empty_cache()
