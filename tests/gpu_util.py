"""Helpers of the GPU parity tests (comparison against the CPU oracle)."""
import sys

import numpy as np


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def same_bits(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


def assert_same_chunks(gpu, osim, where=""):
    assert gpu.nchunks == osim.nchunks
    for c in range(gpu.nchunks):
        g = gpu.export_chunk(c)
        o = osim.chunk(c)
        if g != o:
            raise AssertionError("chunk %d differs %s: gpu %d bytes, oracle %d bytes" % (c, where, len(g), len(o)))
