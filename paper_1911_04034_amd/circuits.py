"""Seeded synthetic circuits and gate records.

This module only builds inputs: arrays of 88-byte gate records with explicit
fp64 matrices, plus seeded random states.  It holds none of the simulator's
arithmetic (no gate application, no truncation, no coding) and imports neither
the HIP library nor the oracle, so both sides can take their inputs from it.

Gate record layout (little-endian, 88 bytes):
    u32 kind, u32 target, u32 target2, u32 reserved, u64 control_mask,
    f64 m[8]
kinds: 0 U1 (general 2x2, row-major u00,u01,u10,u11 as re,im pairs; Eq. (6),
with control_mask for Eq. (7)), 1 DIAG1 (phases d0,d1 on the target bit),
2 DIAG2 (phases p[2*b(target2)+b(target)]), 3 X (Pauli-X, controlled by
control_mask), 4 MCZ (sign flip where all control_mask bits are 1).
Qubit k is bit k of the amplitude index (Eq. (5)).

Benchmarks follow Sec. 5.3 of the paper (Grover, random circuits, QAOA, QFT),
as synthetic generators with the shapes of the workloads listed in
``WORKLOADS``.
"""
from __future__ import annotations

import math

import numpy as np

GATE_DTYPE = np.dtype([
    ("kind", "<u4"), ("target", "<u4"), ("target2", "<u4"), ("reserved", "<u4"),
    ("control_mask", "<u8"), ("m", "<f8", (8,)),
])
assert GATE_DTYPE.itemsize == 88

U1, DIAG1, DIAG2, X, MCZ = 0, 1, 2, 3, 4
KIND_NAMES = {U1: "U1", DIAG1: "DIAG1", DIAG2: "DIAG2", X: "X", MCZ: "MCZ"}

LEVEL_DELTAS = (0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1)


def level_of(delta: float) -> int:
    """Index of a pointwise relative bound among lossless, 1e-5 ... 1e-1."""
    for k, d in enumerate(LEVEL_DELTAS):
        if d == delta:
            return k
    raise ValueError("bound must be one of %r" % (LEVEL_DELTAS,))


# ---------------------------------------------------------------------------
# gate constructors
# ---------------------------------------------------------------------------
def _rec(kind, target=0, target2=0, controls=(), m=None):
    r = np.zeros(1, dtype=GATE_DTYPE)
    r["kind"] = kind
    r["target"] = target
    r["target2"] = target2
    mask = 0
    for c in controls:
        mask |= 1 << int(c)
    r["control_mask"] = mask
    if m is not None:
        r["m"][0, :len(m)] = m
    return r


def u1(q, mat, controls=()):
    """General single-qubit unitary (2x2 complex, row-major) on qubit q."""
    mat = np.asarray(mat, dtype=np.complex128).reshape(2, 2)
    m = [mat[0, 0].real, mat[0, 0].imag, mat[0, 1].real, mat[0, 1].imag,
         mat[1, 0].real, mat[1, 0].imag, mat[1, 1].real, mat[1, 1].imag]
    return _rec(U1, q, 0, controls, m)


def diag1(q, d0, d1, controls=()):
    d0, d1 = complex(d0), complex(d1)
    return _rec(DIAG1, q, 0, controls, [d0.real, d0.imag, d1.real, d1.imag])


def diag2(q1, q2, p):
    p = [complex(v) for v in p]
    return _rec(DIAG2, q1, q2, (), [v for c in p for v in (c.real, c.imag)])


def x(q, controls=()):
    return _rec(X, q, 0, controls)


def mcz(qubits):
    return _rec(MCZ, 0, 0, qubits)


S2 = 1.0 / math.sqrt(2.0)
H_MAT = np.array([[S2, S2], [S2, -S2]], dtype=np.complex128)
SQRTX_MAT = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]])
SQRTY_MAT = 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]])


def h(q):
    return u1(q, H_MAT)


def t(q):
    return diag1(q, 1.0, complex(S2, S2))


def rz(q, theta):
    return diag1(q, complex(math.cos(-theta / 2), math.sin(-theta / 2)),
                 complex(math.cos(theta / 2), math.sin(theta / 2)))


def rx(q, beta):
    c, s = math.cos(beta / 2), math.sin(beta / 2)
    return u1(q, [[c, -1j * s], [-1j * s, c]])


def ry(q, theta):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return u1(q, [[c, -s], [s, c]])


def cphase(control, target, phi):
    return diag1(target, 1.0, complex(math.cos(phi), math.sin(phi)), controls=(control,))


def cz(a, b):
    return mcz((a, b))


def rzz(a, b, gamma):
    """exp(-i gamma Z_a Z_b / 2): phase e^{-i gamma/2} when the bits agree."""
    same = complex(math.cos(-gamma / 2), math.sin(-gamma / 2))
    diff = complex(math.cos(gamma / 2), math.sin(gamma / 2))
    return diag2(a, b, [same, diff, diff, same])


def concat(parts):
    parts = [p for p in parts if len(p)]
    if not parts:
        return np.zeros(0, dtype=GATE_DTYPE)
    return np.concatenate(parts)


# ---------------------------------------------------------------------------
# circuits (Sec. 5.3 benchmark families)
# ---------------------------------------------------------------------------
def random_circuit_small(n=12, depth=20, seed=1):
    """Layers of a seeded qubit permutation; walking it, with p=0.25 the next
    two qubits get CNOT(c, t), else one of {H, T, Rz(theta ~ U[0, 2pi))}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(depth):
        perm = rng.permutation(n)
        k = 0
        while k < n:
            if k + 1 < n and rng.random() < 0.25:
                out.append(x(int(perm[k + 1]), controls=(int(perm[k]),)))
                k += 2
                continue
            which = int(rng.integers(3))
            q = int(perm[k])
            if which == 0:
                out.append(h(q))
            elif which == 1:
                out.append(t(q))
            else:
                out.append(rz(q, float(rng.uniform(0.0, 2 * math.pi))))
            k += 1
    return concat(out)


def grover_marked(n, seed):
    return int(np.random.default_rng(seed).integers(1 << n))


def grover_prefix(n):
    return concat([h(q) for q in range(n)])


def grover_iteration(n, w):
    """Oracle I - 2|w><w| (X on the zero bits of w, MCZ, X) followed by the
    diffusion H X MCZ X H; one iteration equals -G of the textbook."""
    zeros = [q for q in range(n) if not (w >> q) & 1]
    allq = list(range(n))
    parts = [x(q) for q in zeros] + [mcz(allq)] + [x(q) for q in zeros]
    parts += [h(q) for q in allq] + [x(q) for q in allq] + [mcz(allq)]
    parts += [x(q) for q in allq] + [h(q) for q in allq]
    return concat(parts)


def grover(n, iterations, seed):
    w = grover_marked(n, seed)
    it = grover_iteration(n, w)
    return concat([grover_prefix(n)] + [it] * iterations), w


def grover_optimal_iterations(n):
    return int(math.floor(math.pi / 4 * math.sqrt(2.0 ** n)))


def qft_input(n, seed):
    return int(np.random.default_rng(seed).integers(1 << n))


def qft(n, x_in):
    """X on the set bits of x_in, then the textbook QFT ladder from the top
    qubit down, without the final qubit reversal."""
    parts = [x(q) for q in range(n) if (x_in >> q) & 1]
    for j in range(n - 1, -1, -1):
        parts.append(h(j))
        for k in range(j - 1, -1, -1):
            parts.append(cphase(k, j, math.pi / (1 << (j - k))))
    return concat(parts)


def grid_rcs(rows=5, cols=6, depth=20, seed=3):
    """H on every qubit, then per layer an iid choice from {sqrt X, sqrt Y, T}
    on every qubit and CZ on one of four alternating nearest-neighbour edge
    patterns; qubit = cols*row + col."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    out = [h(q) for q in range(n)]
    patterns = []
    for p in range(4):
        edges = []
        if p < 2:
            for r in range(rows):
                for c in range(cols - 1):
                    if c % 2 == p:
                        edges.append((cols * r + c, cols * r + c + 1))
        else:
            for r in range(rows - 1):
                for c in range(cols):
                    if r % 2 == p - 2:
                        edges.append((cols * r + c, cols * (r + 1) + c))
        patterns.append(edges)
    for layer in range(depth):
        for q in range(n):
            which = int(rng.integers(3))
            out.append(u1(q, SQRTX_MAT) if which == 0 else (u1(q, SQRTY_MAT) if which == 1 else t(q)))
        for a, b in patterns[layer % 4]:
            out.append(cz(a, b))
    return concat(out)


def random_regular_graph(n, degree, seed):
    """Configuration model with rejection of self-loops and multi-edges."""
    rng = np.random.default_rng(seed)
    while True:
        stubs = np.repeat(np.arange(n), degree)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        ok = True
        seen = set()
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b or (min(a, b), max(a, b)) in seen:
                ok = False
                break
            seen.add((min(a, b), max(a, b)))
        if ok:
            return sorted(seen)


def qaoa(n=34, p=4, degree=3, seed=5):
    rng = np.random.default_rng(seed)
    edges = random_regular_graph(n, degree, seed)
    gammas = rng.uniform(0.0, math.pi, size=p)
    betas = rng.uniform(0.0, math.pi, size=p)
    out = [h(q) for q in range(n)]
    for layer in range(p):
        out += [rzz(a, b, float(gammas[layer])) for a, b in edges]
        out += [rx(q, float(betas[layer])) for q in range(n)]
    return concat(out), edges


def random_state(n, seed, zero_fraction=0.0):
    """Seeded normalised complex128 state; a fraction of exact zeros."""
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    if zero_fraction > 0:
        psi[rng.random(1 << n) < zero_fraction] = 0
    nrm = np.linalg.norm(psi)
    return psi / (nrm if nrm > 0 else 1.0)


def random_unitary_gates(n, count, seed, with_controls=True):
    """Random gates of every kind on random qubits (test inputs)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(5))
        q = int(rng.integers(n))
        others = [k for k in range(n) if k != q]
        ctrl = ()
        if with_controls and rng.random() < 0.4:
            ctrl = tuple(int(c) for c in rng.choice(others, size=int(rng.integers(1, 3)), replace=False))
        if kind == U1:
            a = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
            qm, _ = np.linalg.qr(a)
            out.append(u1(q, qm, ctrl))
        elif kind == DIAG1:
            ph = rng.uniform(0, 2 * math.pi, size=2)
            out.append(diag1(q, np.exp(1j * ph[0]), np.exp(1j * ph[1]), ctrl))
        elif kind == DIAG2:
            q2 = int(rng.choice(others))
            ph = rng.uniform(0, 2 * math.pi, size=4)
            out.append(diag2(q, q2, np.exp(1j * ph)))
        elif kind == X:
            out.append(x(q, ctrl))
        else:
            qs = (q,) + ctrl
            out.append(mcz(qs))
    return concat(out)


# ---------------------------------------------------------------------------
# named workloads (shapes of the benchmark configurations)
# ---------------------------------------------------------------------------
WORKLOADS = {
    "rand12": dict(n=12, block_log2=8, level=1,
                   doc="12-qubit seeded random circuit of depth 20 over {H, T, Rz, CNOT}, 2^8-amplitude blocks"),
    "grover24": dict(n=24, block_log2=16, level=1,
                     doc="24-qubit Grover, seeded marked index, 2^16-amplitude blocks, bound 1e-5"),
    "qft24": dict(n=24, block_log2=16, level=1,
                  doc="24-qubit QFT of a seeded basis state, 2^16-amplitude blocks, bound 1e-5"),
    "grid30": dict(n=30, block_log2=20, level=2,
                   doc="30-qubit 5x6 grid random circuit, depth 20, 2^20-amplitude blocks, bound 1e-4"),
    "grover36": dict(n=36, block_log2=20, level=1,
                     doc="36-qubit Grover, 8 iterations, 2^20-amplitude blocks, bound 1e-5"),
    "qaoa34": dict(n=34, block_log2=20, level=2,
                   doc="34-qubit QAOA on a seeded 3-regular graph, p=4"),
}


def biased_local(n=16, block_log2=8, depth=12, seed=41):
    """A state whose block weights are uneven and stay so: Ry(theta) with
    theta ~ U[0.12 pi, 0.3 pi] on every block-index qubit (weight of a block =
    product of cos^2 / sin^2 factors), then `depth` layers of the
    random_circuit_small pattern on the in-block qubits, Rz on every
    block-index qubit and CZ on a seeded pair of them (diagonal there: no
    weight moves between blocks)."""
    rng = np.random.default_rng(seed)
    hi = list(range(block_log2, n))
    out = [ry(q, float(rng.uniform(0.12 * math.pi, 0.3 * math.pi))) for q in hi]
    for layer in range(depth):
        local = random_circuit_small(block_log2, 1, int(rng.integers(1 << 30)))
        out.append(local)
        out += [rz(q, float(rng.uniform(0.0, 2 * math.pi))) for q in hi]
        if len(hi) >= 2:
            a, b = rng.choice(len(hi), size=2, replace=False)
            out.append(cz(hi[int(a)], hi[int(b)]))
    return concat(out)
