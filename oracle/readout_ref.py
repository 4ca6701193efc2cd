"""Plain reference of the readout calls: sampling without collapse and the
overlap of two states.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product
package.  Python integers and numpy float64 over states decoded by the C
oracle.

Sampling draws basis index i with probability |a_i|^2 / sum |a|^2 (the
measurement the paper's simulations end with, Sec. 2): shot k takes
u_k = (output k of SplitMix64 seeded with `seed`) >> 11, times 2^-53, and
t = u_k * total; the chunk is the first whose running squared norm (chunk
order) exceeds t, the amplitude the first in that chunk whose running |a|^2
(index order) exceeds the remainder of t, or the chunk's last nonzero
amplitude when rounding runs past its end.
"""
from __future__ import annotations

import bisect

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(seed: int, k: int) -> int:
    """Output k (from 0) of SplitMix64 (Steele, Lea and Flood, 2014) whose
    state starts at `seed`: state advances by the golden-ratio increment,
    then two xor-shift-multiply rounds and a final xor-shift."""
    z = (seed + (k + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def sample(psi, amps_per_chunk: int, seed: int, shots: int) -> np.ndarray:
    """psi: complex128 state (decoded); returns uint64 indices."""
    psi = np.asarray(psi, dtype=np.complex128)
    x = psi.view(np.float64)
    nch = psi.size // amps_per_chunk
    norms = []
    for c in range(nch):
        acc = 0.0
        for v in x[2 * c * amps_per_chunk:2 * (c + 1) * amps_per_chunk]:
            acc += float(v) * float(v)
        norms.append(acc)
    cdf, run, last_nz = [], 0.0, 0
    for c, p in enumerate(norms):
        if p > 0.0:
            last_nz = c
        run += p
        cdf.append(run)
    total = run
    out = np.zeros(shots, dtype=np.uint64)
    for k in range(shots):
        u = (splitmix64(seed, k) >> 11) * 2.0 ** -53
        t = u * total
        c = bisect.bisect_right(cdf, t)
        if c >= nch:
            c = last_nz
        rest = t - (cdf[c - 1] if c else 0.0)
        acc, pick, nz = 0.0, None, 0
        for i in range(amps_per_chunk):
            re = float(x[2 * (c * amps_per_chunk + i)])
            im = float(x[2 * (c * amps_per_chunk + i) + 1])
            p = re * re + im * im
            if p > 0.0:
                nz = i
            acc += p
            if acc > rest:
                pick = i
                break
        out[k] = c * amps_per_chunk + (pick if pick is not None else nz)
    return out


def overlap(a, b) -> complex:
    """<a|b> = sum conj(a_i) b_i."""
    return complex(np.vdot(np.asarray(a, dtype=np.complex128), np.asarray(b, dtype=np.complex128)))
