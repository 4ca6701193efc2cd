"""Host logic of the benchmark: the timed windows are cut at the boundaries
of the passes the library forms (fused runs of single-chunk gates, chunk-
group runs on up to two or three chunk-index qubits), so that no step splits
a pass.  CPU only."""
import numpy as np

import bench
from paper_1911_04034_amd import circuits as cc


def passes_of(gates, cb, group_bits):
    """Reference grouping written from the run rules: consecutive single-chunk
    gates (diagonal, MCZ, in-chunk targets) form one pass of up to 64;
    consecutive chunk-pair gates form one pass while their distinct targets
    number at most group_bits."""
    out = []
    for i, g in enumerate(gates):
        k, t, cm = int(g["kind"]), int(g["target"]), int(g["control_mask"])
        if k in (cc.DIAG1, cc.DIAG2, cc.MCZ) or t < cb:
            kind = "single"
        elif k == cc.X and (cm & ((1 << cb) - 1)) == 0:
            kind = "permute"
        else:
            kind = "pair"
        if out and out[-1][0] == kind and len(out[-1][1]) < 64 and kind != "permute":
            if kind == "single" or len(out[-1][2] | {t}) <= group_bits:
                out[-1][1].append(i)
                if kind == "pair":
                    out[-1][2].add(t)
                continue
        out.append((kind, [i], {t} if kind == "pair" else set()))
    return [p[1] for p in out]


def test_windows_never_split_a_pass_and_cover_the_circuit():
    gates = cc.qaoa(34, 4, 3, 5)[0]
    cb = 10
    for group_bits in (2, 3):
        ref = passes_of(gates, cb, group_bits)
        for nwin in (1, 4, 25, 200):
            wins = bench.pass_windows(gates, cb, nwin, True, group_bits=group_bits)
            assert sum(len(w) for w in wins) == len(gates)
            assert np.array_equal(np.concatenate(wins), gates)
            # every window boundary is a pass boundary
            starts = {p[0] for p in ref}
            pos = 0
            for w in wins:
                assert pos in starts
                pos += len(w)
            assert len(wins) == min(nwin, len(ref))


def test_qaoa34_pass_counts():
    """A QAOA-34 layer: the 51 Rzz and the 10 in-chunk mixers are one pass,
    the 24 chunk-index mixers 12 passes on two qubits or 8 on three."""
    gates = cc.qaoa(34, 4, 3, 5)[0]
    layer = gates[34 + 51 + 34:34 + 2 * (51 + 34)]
    for group_bits, npair in ((2, 12), (3, 8)):
        ps = passes_of(layer, 10, group_bits)
        assert len(ps) == 1 + npair
        assert len(bench.pass_windows(layer, 10, 1000, True, group_bits=group_bits)) == 1 + npair
