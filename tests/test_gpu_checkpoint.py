"""Checkpoint and resume (Sec. 3.5): a run interrupted after k gates, saved
(compressed chunks + ledger), reloaded into a fresh state and continued,
ends with the bytes and ledger of the uninterrupted run, which are the
oracle's."""
import ctypes

import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say

pytestmark = pytest.mark.gpu

LEDGER = ("compressed_bytes", "gates_applied", "lossy_steps", "min_compressed", "max_compressed", "level",
          "fidelity_lower_bound")


def run_interrupted(tmp_path, n, bl, mode, level, budget, gates, cut, **kw):
    from paper_1911_04034_amd import qcz
    a = qcz.State(n, bl, mode=mode, level=level, budget=budget, pool_bytes=64 << 20, **kw)
    rc_a, done_a = a.try_apply(gates)
    b = qcz.State(n, bl, mode=mode, level=level, budget=budget, pool_bytes=64 << 20, **kw)
    assert b.apply(gates[:cut]) == cut
    path = str(tmp_path / "ckpt.npz")
    b.save(path)
    c = qcz.State.load(path, pool_bytes=64 << 20)
    assert all(c.footprint()[k] == b.footprint()[k] for k in LEDGER)
    rc_c, done_c = c.try_apply(gates[cut:])
    return a, (rc_a, done_a), c, (rc_c, done_c)


@pytest.mark.parametrize("mode,level", [(oq.MODE_LOSSLESS, 0), (oq.MODE_FIXED, 2)])
def test_resume_continues_bytes_and_ledger(tmp_path, mode, level):
    n, bl = 12, 8
    gates = cc.concat([cc.grover_prefix(n), cc.random_circuit_small(n, depth=12, seed=41)])
    cut = len(gates) // 2
    say("checkpoint mode=%d level=%d at gate %d of %d" % (mode, level, cut, len(gates)))
    a, (rc_a, _), c, (rc_c, _) = run_interrupted(tmp_path, n, bl, mode, level, 0, gates, cut, batch=16)
    assert rc_a == 0 and rc_c == 0
    assert_same_chunks(c, a_as_oracle(a), "after resume")
    fa, fc = a.footprint(), c.footprint()
    for k in LEDGER:
        assert fc[k] == fa[k], k
    o = oq.Sim(n, bl, mode, level, 0)
    o.apply(gates)
    assert_same_chunks(c, o, "against the oracle")
    assert fc["fidelity_lower_bound"] == pytest.approx(o.footprint()["fidelity_lower_bound"], rel=1e-12)


def test_resume_adaptive_takes_the_same_decisions(tmp_path):
    n, bl = 12, 8
    gates = cc.random_circuit_small(n, depth=20, seed=21)
    ref = oq.Sim(n, bl, oq.MODE_LOSSLESS)
    peak = 0
    for k in range(len(gates)):
        ref.apply(gates[k:k + 1])
        peak = max(peak, ref.footprint()["compressed_bytes"])
    budget = int(0.6 * peak)
    o = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    rc_o = o.apply(gates)
    assert rc_o >= 0
    # cut a few gates after the level has first risen
    probe = oq.Sim(n, bl, oq.MODE_ADAPTIVE, 0, budget)
    cut = None
    for k in range(len(gates)):
        probe.apply(gates[k:k + 1])
        if probe.footprint()["level"] > 0:
            cut = k + 4
            break
    assert cut is not None and cut < len(gates)
    say("adaptive checkpoint at gate %d, budget %d" % (cut, budget))
    a, (rc_a, _), c, (rc_c, _) = run_interrupted(tmp_path, n, bl, oq.MODE_ADAPTIVE, 0, budget, gates, cut, batch=8)
    assert rc_a == 0 and rc_c == 0
    fo, fc = o.footprint(), c.footprint()
    assert fc["level"] == fo["level"] > 0
    assert fc["compressed_bytes"] == fo["compressed_bytes"]
    assert fc["lossy_steps"] == fo["lossy_steps"]
    assert_same_chunks(c, o, "adaptive resume against the oracle")


def test_resume_rejects_mismatches():
    from paper_1911_04034_amd import qcz
    n, bl = 10, 7
    s = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=1, pool_bytes=16 << 20)
    s.apply(cc.grover_prefix(n))
    fp = qcz.Footprint()
    s._check(s._lib.qcz_footprint(s._h, ctypes.byref(fp)), "qcz_footprint")
    L = s._lib
    fresh = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=1, pool_bytes=16 << 20)
    # streams not imported: the compressed size differs from the record
    assert L.qcz_resume(fresh._h, ctypes.byref(fp)) == -5
    bad = qcz.Footprint.from_buffer_copy(bytes(fp))
    bad.fidelity_lower_bound = 1.5
    assert L.qcz_resume(s._h, ctypes.byref(bad)) == -1
    other = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=3, pool_bytes=16 << 20)
    assert L.qcz_resume(other._h, ctypes.byref(fp)) == -1
    perblock = qcz.State(n, bl, mode=qcz.MODE_PERBLOCK, level=1, pool_bytes=16 << 20)
    fp0 = qcz.Footprint()
    perblock._check(L.qcz_footprint(perblock._h, ctypes.byref(fp0)), "qcz_footprint")
    assert L.qcz_resume(perblock._h, ctypes.byref(fp0)) == -5
    # the state itself is untouched by the rejected calls
    assert L.qcz_resume(s._h, ctypes.byref(fp)) == 0


def a_as_oracle(a):
    """The uninterrupted GPU run viewed through the comparison helper."""
    class View:
        nchunks = a.nchunks

        @staticmethod
        def chunk(c):
            return a.export_chunk(c)
    return View


def test_state_image_matches_chunk_exports():
    """The one-copy image holds every chunk's stream at its 16-byte offset,
    zero up to the boundary; importing it into a fresh state gives the same
    chunks, and a malformed image is refused without touching the state."""
    import numpy as np
    from paper_1911_04034_amd import qcz
    n, bl = 12, 8
    s = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=2, pool_bytes=64 << 20)
    s.apply(cc.concat([cc.grover_prefix(n), cc.random_circuit_small(n, depth=8, seed=2)]))
    image, sizes = s.export_state()
    off = 0
    for c in range(s.nchunks):
        blob = s.export_chunk(c)
        assert len(blob) == sizes[c]
        assert image[off:off + len(blob)].tobytes() == blob
        unit = (len(blob) + 15) // 16 * 16
        assert not image[off + len(blob):off + unit].any()
        off += unit
    assert off == image.size
    t = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=2, pool_bytes=64 << 20)
    before = [t.export_chunk(c) for c in range(t.nchunks)]
    bad = image.copy()
    bad[0:4] = 0xFF
    with pytest.raises(qcz.QczError):
        t.import_state(bad, sizes)
    assert [t.export_chunk(c) for c in range(t.nchunks)] == before
    t.import_state(image, sizes)
    assert_same_chunks(t, a_as_oracle(s), "after the image import")
    assert t.footprint()["compressed_bytes"] == s.footprint()["compressed_bytes"]


def test_checkpoint_full_size_grover24(tmp_path):
    """At the benchmark shape (16384 chunks) a checkpoint taken after one
    Grover iteration reloads the same streams and ledger, and both states
    continue identically."""
    import time
    import numpy as np
    from paper_1911_04034_amd import qcz
    n, bl = 24, 16
    w = cc.grover_marked(n, 2)
    it = cc.grover_iteration(n, w)
    a = qcz.State(n, bl, mode=qcz.MODE_FIXED, level=1, pool_bytes=2 << 30, batch=128)
    a.apply(cc.grover_prefix(n))
    a.apply(it)
    path = str(tmp_path / "grover24.npz")
    t0 = time.perf_counter()
    a.save(path)
    b = qcz.State.load(path, pool_bytes=2 << 30)
    say("grover24 checkpoint save + load %.2f s" % (time.perf_counter() - t0))
    assert np.array_equal(a.chunk_sizes(), b.chunk_sizes())
    assert all(a.footprint()[k] == b.footprint()[k] for k in LEDGER)
    rng = np.random.default_rng(3)
    for c in rng.choice(a.nchunks, size=64, replace=False):
        assert a.export_chunk(int(c)) == b.export_chunk(int(c))
    a.apply(it)
    b.apply(it)
    assert np.array_equal(a.chunk_sizes(), b.chunk_sizes())
    for c in rng.choice(a.nchunks, size=64, replace=False):
        assert a.export_chunk(int(c)) == b.export_chunk(int(c))
    assert all(a.footprint()[k] == b.footprint()[k] for k in LEDGER)
