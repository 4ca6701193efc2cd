"""The C-ABI library loads and exports every function include/qcz.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qcz.h")
LIB = os.path.join(ROOT, "paper_1911_04034_amd", "libqcz.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(qcz_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("qcz_create", "qcz_apply_gates", "qcz_read_amplitudes", "qcz_footprint", "qcz_destroy",
                     "qcz_export_chunk", "qcz_encode_chunks", "qcz_decode_chunks"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcz.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcz.so not built")
def test_binding_lists_match_header():
    from paper_1911_04034_amd import qcz
    assert sorted(qcz.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcz.so not built")
def test_host_only_calls():
    from paper_1911_04034_amd import qcz
    L = qcz.load()
    assert L.qcz_chunk_cap(2048) == 4 + 512 + 8 * 2048
    cfg = qcz.Config(12, 8, 0, 0, 0, 0, 0, 0, 0)
    assert L.qcz_pool_bytes_min(ctypes.byref(cfg)) > 0
    bad = qcz.Config(3, 8, 0, 0, 0, 0, 0, 0, 0)
    assert L.qcz_pool_bytes_min(ctypes.byref(bad)) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libqcz.so not built")
def test_block_cache_pool_and_stats_layout():
    """The block cache's key table (12 bytes per chunk), role and key arrays
    (4 + 8 bytes per job) and the copy kernel's 1024 per-workgroup sums (56 bytes each)
    come out of the pool; the stats record ends with the cache counters as
    the header lays them out."""
    from paper_1911_04034_amd import qcz
    L = qcz.load()
    n, bl = 20, 12
    plain = L.qcz_pool_bytes_min(ctypes.byref(qcz.Config(n, bl, 1, 1, 0, 0, 0, 0, 0)))
    cached = L.qcz_pool_bytes_min(ctypes.byref(qcz.Config(n, bl, 1, 1, 0, qcz.FLAG_CACHE, 0, 0, 0)))
    nchunks = 1 << (n - 10)
    need = 12 * nchunks + 12 * (nchunks // 2) + 1024 * 56
    assert need <= cached - plain <= need + 5 * 256
    assert qcz.Stats.cache_on.offset == qcz.Stats.cache_hits.offset + 8
    assert ctypes.sizeof(qcz.Stats) == qcz.Stats.kind_bytes.offset + 24 == qcz.Stats.sweep_gates.offset + 80 \
        == qcz.Stats.range_launches.offset + 88 == qcz.Stats.reserved.offset + 92


def test_profile_summaries_parse():
    """The bench reads its traffic and VALU-busy figures from the committed
    rocprofv3 summaries, each tagged with the kernel source hash it was
    taken with."""
    from paper_1911_04034_amd import profile_summary as ps
    prof = os.path.join(ROOT, "profiles")
    t_bytes, t_hash = ps.read_traffic(os.path.join(prof, "traffic_fused_kernel_grover24_qft24.txt"))
    busy, b_hash = ps.read_valu_busy(os.path.join(prof, "counters_fused_kernel_qft24_grover24.txt"))
    assert t_bytes is not None and t_bytes > 0 and len(t_hash) == 16
    assert set(busy) == {"qft24", "grover24"} and all(0.0 < v <= 1.0 for v in busy.values())
    assert len(b_hash) == 16
