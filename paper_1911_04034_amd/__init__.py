"""MI355X-native compressed full-state quantum circuit simulation.

The hot path (decompress -> apply gate -> recompress over a chunked,
compressed complex128 state) runs in hand-written HIP kernels built into
``libqcz.so``; ``qcz.py`` is the thin ctypes binding to its C ABI
(``include/qcz.h``).  ``circuits.py`` builds seeded gate lists.

Importing this package does not load the HIP library; ``qcz.load()`` does,
and raises if it is missing.
"""
__all__ = ["circuits", "qcz"]
