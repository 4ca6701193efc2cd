"""Plain reference of the per-block statistics, per-level sizes, level labels
and budget projection used by the learned level selector.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product
package.  numpy in float64 plus the C oracle's codec.

The selector generalises the variable error bound of Sec. 3.7 from one level
for the whole state to one level per block, and keeps the Sec. 3.8 argument:
if block b is truncated at relative error delta_b per value, one step keeps
the fidelity at least 1 - sum_b w_b delta_b with w_b the block's share of the
squared norm.  Levels are chosen for a window of gates, during which weight
moves between blocks: gates whose target is a block-index qubit (mask M of
such bits) only move it inside the cosets {b' : b' & ~M == b & ~M}, whose
total weight W_c the window's unitary gates conserve.  The per-step budget is
therefore sum over cosets of W_c * max_{b in c} delta_b <= beta, which holds
at every gate of the window and gives at least the Eq. (11) product of a
uniform bound beta.

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
   f15 (number of block-index bits in the window's mixing mask) / 16
"""
from __future__ import annotations

import math

import numpy as np

from oracle import qcz_oracle as oq

DELTA = [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]
SLACK = 1.0 + 2.0 ** -20   # feasibility: sum_b w_b delta_b <= beta * SLACK


def _pad4(n):
    return (n + 3) & ~3


def block_features(sim, levels, beta, mask=0):
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
        f[15] = bin(mask).count("1") / 16.0
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


def cosets(nblocks, mask):
    """Coset id of every block (b & ~mask) and the sorted distinct ids."""
    ids = np.arange(nblocks, dtype=np.int64) & ~np.int64(mask)
    return ids, sorted(set(int(x) for x in ids))


def coset_weights(w, mask):
    ids, order = cosets(len(w), mask)
    W = {c: 0.0 for c in order}
    for b in range(len(w)):
        W[int(ids[b])] += float(w[b])
    return ids, order, W


def _weighted(levels, w, mask=0):
    """sum over cosets (increasing id) of W_c * delta(max level in c)."""
    ids, order, W = coset_weights(w, mask)
    top = {c: 0 for c in order}
    for b in range(len(w)):
        top[int(ids[b])] = max(top[int(ids[b])], int(levels[b]))
    tot = 0.0
    for c in order:
        tot += W[c] * DELTA[top[c]]
    return tot


def _capped(S, b, cap):
    """Level <= cap with the fewest bytes for block b (lowest on ties)."""
    best = 0
    for lev in range(1, cap + 1):
        if S[b, lev] < S[b, best]:
            best = lev
    return best


def label_levels(S, w, beta, mask=0):
    """Per coset c a cap level minimising (bytes of its blocks, each at its
    smallest level <= cap) + lambda * W_c * delta(cap), lowest cap on ties,
    for the smallest lambda among 0 and the values where some coset's choice
    changes whose caps satisfy sum_c W_c delta(cap_c) <= beta * SLACK; each
    block then takes its smallest level under its coset's cap."""
    nb = len(w)
    ids, order, W = coset_weights(w, mask)
    members = {c: [b for b in range(nb) if int(ids[b]) == c] for c in order}
    cost = {c: [float(sum(int(S[b, _capped(S, b, cap)]) for b in members[c])) for cap in range(6)] for c in order}
    lim = beta * SLACK
    cands = set()
    for c in order:
        if W[c] <= 0.0:
            continue
        for lo in range(6):
            for hi in range(lo + 1, 6):
                d = cost[c][lo] - cost[c][hi]
                if d > 0.0:
                    cands.add(d / (W[c] * (DELTA[hi] - DELTA[lo])))
    caps = None
    for lam in [0.0] + sorted(cands):
        cp = {}
        for c in order:
            best, bc = 0, None
            for cap in range(6):
                v = cost[c][cap] + lam * (W[c] * DELTA[cap])
                if bc is None or v < bc:
                    best, bc = cap, v
            cp[c] = best
        tot = 0.0
        for c in order:
            tot += W[c] * DELTA[cp[c]]
        if tot <= lim:
            caps = cp
            break
    L = np.zeros(nb, dtype=np.uint8)
    if caps is None:
        return L
    for b in range(nb):
        L[b] = _capped(S, b, caps[int(ids[b])])
    return L


def project_levels(levels, w, beta, mask=0):
    """While the coset budget is exceeded, take the coset with the largest
    W_c * delta(max level) (lowest id on ties) and lower by one every block
    of it at that max level."""
    L = np.array(levels, dtype=np.uint8).copy()
    ids, order, W = coset_weights(w, mask)
    lim = beta * SLACK
    while _weighted(L, w, mask) > lim:
        best, bv, btop = -1, -1.0, 0
        for c in order:
            top = max(int(L[b]) for b in range(len(w)) if int(ids[b]) == c)
            v = W[c] * DELTA[top]
            if v > bv:
                best, bv, btop = c, v, top
        for b in range(len(w)):
            if int(ids[b]) == best and int(L[b]) == btop:
                L[b] -= 1
    return L


def rule_level(beta):
    """The loosest level whose delta is at most beta (0 = lossless)."""
    r = 0
    for lev in range(1, 6):
        if DELTA[lev] <= beta:
            r = lev
    return r


def select_from_network(levels, w, beta, mask=0):
    """The selector's levels from the network's per-block choice: each raised
    to at least the rule's level (one bound for every block, delta <= beta,
    already meets the budget), then projected onto the coset budget."""
    floor = rule_level(beta)
    L = np.maximum(np.asarray(levels, dtype=np.uint8), np.uint8(floor))
    return project_levels(L, w, beta, mask)
