"""Plain reference of the per-block statistics, per-level sizes, level labels
and budget projection used by the learned level selector.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product
package.  numpy in float64 plus the C oracle's codec.

The selector generalises the variable error bound of Sec. 3.7 from one level
for the whole state to one level per block, and keeps the Sec. 3.8 argument:
if block b is truncated at relative error delta_b per value, one step keeps
the fidelity at least 1 - sum_b w_b delta_b with w_b the block's share of the
squared norm.  A per-step budget beta on sum_b w_b delta_b therefore gives the
same Eq. (11) product as a uniform bound beta.

Block features (16 per block; M = 2^(block_log2+1) stored doubles of block b
in interleaved re/im order, C doubles per chunk, previous value of a chunk's
first value = +0.0, u = IEEE-754 bits, e = biased exponent of a nonzero
value):
   f0  log2(max(n2_b * nblocks, 2^-60)) / 64, n2_b = sum of squares
   f1  1 - (#nonzero values) / M
   f2  (mean e over nonzero values - 1023) / 64        (0 if none)
   f3  (max e - min e) / 64                            (0 if none)
   f4  #{u_i >> 56 == u_prev >> 56} / M
   f5  #{u_i >> 48 == u_prev >> 48} / M
   f6  #{u_i >> 40 == u_prev >> 40} / M
   f7  #{sign bit differs from the previous value's} / M
   f8  fraction of the block's chunks stored as two constants
   f9  padded stream bytes of the block / (16 * 2^block_log2)
   f10 current level of the block / 5
   f11 (max e - 1023) / 64                            (-17 if none)
   f12 max(log10(beta), -20) / 5
   f13 log2(2^(n+4) / padded stream bytes of the state) / 16
   f14 log2(nblocks) / 16
   f15 block_log2 / 32
"""
from __future__ import annotations

import math

import numpy as np

from oracle import qcz_oracle as oq

DELTA = [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]
SLACK = 1.0 + 2.0 ** -20   # feasibility: sum_b w_b delta_b <= beta * SLACK


def _pad4(n):
    return (n + 3) & ~3


def block_features(sim, levels, beta):
    """Features (nblocks x 16, float64) and n2_b (nblocks) of an oracle Sim."""
    n, bl, cb, C = sim.n, sim.block_log2, sim.cb, sim.C
    nblocks = 1 << (n - bl)
    cpb = 1 << (bl - cb)
    M = 2 << bl
    streams = [sim.chunk(c) for c in range(sim.nchunks)]
    live = sum(_pad4(len(s)) for s in streams)
    F = np.zeros((nblocks, 16), dtype=np.float64)
    n2 = np.zeros(nblocks, dtype=np.float64)
    for b in range(nblocks):
        acc = 0.0
        nz = 0
        esum = 0
        emax, emin = -1, 4096
        eq8 = eq16 = eq24 = sgn = 0
        const2 = 0
        nbytes = 0
        for k in range(cpb):
            s = streams[b * cpb + k]
            nbytes += _pad4(len(s))
            if int.from_bytes(s[:4], "little") & 3 == 1:
                const2 += 1
            x = oq.decode_chunk(s, C)
            u = x.view(np.uint64)
            for i in range(C):
                acc += float(x[i]) * float(x[i])
            prev = np.concatenate([np.zeros(1, np.uint64), u[:-1]])
            nzm = x != 0.0
            nz += int(nzm.sum())
            e = ((u >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64)[nzm]
            if e.size:
                esum += int(e.sum())
                emax = max(emax, int(e.max()))
                emin = min(emin, int(e.min()))
            eq8 += int(np.sum((u >> np.uint64(56)) == (prev >> np.uint64(56))))
            eq16 += int(np.sum((u >> np.uint64(48)) == (prev >> np.uint64(48))))
            eq24 += int(np.sum((u >> np.uint64(40)) == (prev >> np.uint64(40))))
            sgn += int(np.sum((u >> np.uint64(63)) != (prev >> np.uint64(63))))
        n2[b] = acc
        f = F[b]
        f[0] = math.log2(max(acc * nblocks, 2.0 ** -60)) / 64.0
        f[1] = 1.0 - nz / M
        f[2] = (esum / nz - 1023.0) / 64.0 if nz else 0.0
        f[3] = (emax - emin) / 64.0 if nz else 0.0
        f[4], f[5], f[6], f[7] = eq8 / M, eq16 / M, eq24 / M, sgn / M
        f[8] = const2 / cpb
        f[9] = nbytes / (16.0 * (1 << bl))
        f[10] = levels[b] / 5.0
        f[11] = (emax - 1023.0) / 64.0 if nz else -17.0
        f[12] = max(math.log10(beta), -20.0) / 5.0 if beta > 0 else -4.0
        f[13] = math.log2((2.0 ** (n + 4)) / live) / 16.0
        f[14] = math.log2(nblocks) / 16.0
        f[15] = bl / 32.0
    return F, n2


def block_level_sizes(sim):
    """Padded bytes of each block re-encoded at each of the six levels."""
    n, bl, cb, C = sim.n, sim.block_log2, sim.cb, sim.C
    nblocks = 1 << (n - bl)
    cpb = 1 << (bl - cb)
    S = np.zeros((nblocks, 6), dtype=np.uint64)
    for c in range(sim.nchunks):
        x = oq.decode_chunk(sim.chunk(c), C)
        for lev in range(6):
            S[c // cpb, lev] += _pad4(len(oq.encode_chunk(x, lev)))
    return S


def _weighted(levels, w):
    tot = 0.0
    for b in range(len(w)):
        tot += float(w[b]) * DELTA[int(levels[b])]
    return tot


def _argmin_levels(S, w, lam):
    L = np.zeros(len(w), dtype=np.uint8)
    for b in range(len(w)):
        best, bestc = 0, None
        for lev in range(6):
            c = float(S[b, lev]) + lam * (float(w[b]) * DELTA[lev])
            if bestc is None or c < bestc:
                best, bestc = lev, c
        L[b] = best
    return L


def breakpoints(S, w):
    """Every lambda at which some block's Lagrangian choice can change."""
    out = set()
    for b in range(len(w)):
        if w[b] <= 0.0:
            continue
        for lo in range(6):
            for hi in range(lo + 1, 6):
                ds = float(S[b, lo]) - float(S[b, hi])
                if ds > 0.0:
                    out.add(ds / (float(w[b]) * (DELTA[hi] - DELTA[lo])))
    return sorted(out)


def label_levels(S, w, beta):
    """Per-block level minimising size + lambda * w_b * delta, with the
    smallest lambda among {0} and the breakpoints whose choice meets the
    budget; ties between levels go to the tighter one."""
    lim = beta * SLACK
    for lam in [0.0] + breakpoints(S, w):
        L = _argmin_levels(S, w, lam)
        if _weighted(L, w) <= lim:
            return L
    return np.zeros(len(w), dtype=np.uint8)


def project_levels(levels, w, beta):
    """Tighten one level at a time the block with the largest w_b delta_b
    (lowest index on ties) until sum_b w_b delta_b <= beta * SLACK."""
    L = np.array(levels, dtype=np.uint8).copy()
    lim = beta * SLACK
    while _weighted(L, w) > lim:
        best, bv = -1, -1.0
        for b in range(len(w)):
            v = float(w[b]) * DELTA[int(L[b])]
            if v > bv:
                best, bv = b, v
        L[best] -= 1
    return L
