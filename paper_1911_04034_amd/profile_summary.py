"""Readers of the rocprofv3 summaries under profiles/ that the benchmark
reports beside its own timing (counter-measured traffic and VALU-busy
fraction of the fused kernel), and the hash of the device code that tells
whether a summary still describes the current kernels.  The summaries are
written by profile_summary.py at the repository root."""
from __future__ import annotations

import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "qcz_kernels.hip")


def kernel_hash() -> str:
    """Hash of the device code (the file up to its host launchers)."""
    src = open(KERNEL_SRC, "rb").read()
    cut = src.find(b"// host launchers")
    return hashlib.sha256(src[:cut] if cut > 0 else src).hexdigest()[:16]


def read_valu_busy(path):
    """({workload: VALU busy per SIMD}, kernel hash) from a counters summary, or ({}, None)."""
    if not os.path.exists(path):
        return {}, None
    busy, h, cur = {}, None, None
    for line in open(path):
        if line.startswith("# kernel source sha256[:16]:"):
            h = line.rsplit(":", 1)[1].strip()
        elif line.startswith("workload "):
            cur = line.split()[1]
        elif cur and line.strip().startswith("VALU busy per SIMD"):
            busy[cur] = float(line.split()[-1])
    return busy, h


def read_traffic(path):
    """(bytes per dispatch, kernel hash) from a traffic summary, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    try:
        return float(vals["traffic_bytes_per_dispatch"]), vals["kernel_source_sha256_16"]
    except (KeyError, ValueError):
        return None, None
