"""Uncompressed fp64 state-vector simulation with torch on the device, for
measuring the fidelity of a compressed run (Eq. (9): |<psi_ideal|psi_sim>|).

A test aid, not part of the compressed path (only tests import it): it holds the
full 2^n complex128 vector (16 GiB at 30 qubits) and applies the same gate
records with tensor views over the qubit dimensions.  Qubit q is bit q of
the amplitude index, i.e. dimension n - 1 - q of the [2] * n view.
"""
from __future__ import annotations

import numpy as np

U1, DIAG1, DIAG2, X, MCZ = 0, 1, 2, 3, 4


def _torch():
    import torch
    return torch


def zero_state(n: int, device="cuda"):
    torch = _torch()
    psi = torch.zeros(1 << n, dtype=torch.complex128, device=device)
    psi[0] = 1.0
    return psi


def _controlled_view(v, n: int, controls):
    """Sub-view of the [2]*n view where every control bit is 1, and a map
    from qubit to the dimension it has in that sub-view."""
    dims = {q: n - 1 - q for q in range(n)}
    for c in sorted(controls, key=lambda q: -(n - 1 - q)):   # highest dimension first keeps others valid
        d = n - 1 - c
        v = v.select(d, 1)
        for q in range(n):
            if dims[q] is not None and dims[q] > d:
                dims[q] -= 1
        dims[c] = None
    return v, dims


def apply_gate(psi, n: int, g):
    """Apply one gate record (circuits.GATE_DTYPE) to psi in place."""
    torch = _torch()
    kind = int(g["kind"])
    q, q2 = int(g["target"]), int(g["target2"])
    cm = int(g["control_mask"])
    m = [float(x) for x in g["m"]]
    controls = [b for b in range(n) if (cm >> b) & 1]
    v = psi.view([2] * n)
    if kind == MCZ:
        sub, _ = _controlled_view(v, n, controls)
        sub.mul_(-1.0)
        return
    sub, dims = _controlled_view(v, n, controls)
    if kind in (U1, X):
        d = dims[q]
        a0 = sub.select(d, 0)
        a1 = sub.select(d, 1)
        if kind == X:
            t = a0.clone()
            a0.copy_(a1)
            a1.copy_(t)
            return
        u00, u01, u10, u11 = (complex(m[0], m[1]), complex(m[2], m[3]), complex(m[4], m[5]), complex(m[6], m[7]))
        n0 = a0 * u00 + a1 * u01
        n1 = a0 * u10 + a1 * u11
        a0.copy_(n0)
        a1.copy_(n1)
        return
    if kind == DIAG1:
        d = dims[q]
        sub.select(d, 0).mul_(complex(m[0], m[1]))
        sub.select(d, 1).mul_(complex(m[2], m[3]))
        return
    if kind == DIAG2:
        d1, d2 = dims[q], dims[q2]
        for b2 in (0, 1):
            for b1 in (0, 1):
                p = complex(m[2 * (2 * b2 + b1)], m[2 * (2 * b2 + b1) + 1])
                if d1 > d2:
                    sub.select(d1, b1).select(d2, b2).mul_(p)
                else:
                    sub.select(d2, b2).select(d1, b1).mul_(p)
        return
    raise ValueError("unknown gate kind %d" % kind)


def run(gates, n: int, psi=None):
    """psi (default |0...0>) after the gate list."""
    if psi is None:
        psi = zero_state(n)
    for g in np.asarray(gates):
        apply_gate(psi, n, g)
    return psi


def overlap_with_compressed(psi_ref, state, chunks_per_call: int = 4096):
    """<psi_ref|psi_sim> and |psi_sim|^2, decoding the compressed state in
    slices (complex, float)."""
    torch = _torch()
    C = state.C
    ov = 0j
    n2 = 0.0
    buf = torch.empty(chunks_per_call * C, dtype=torch.float64, device=psi_ref.device)
    amps = C // 2
    for c0 in range(0, state.nchunks, chunks_per_call):
        m = min(chunks_per_call, state.nchunks - c0)
        state.decode_to(c0, m, buf[:m * C])
        sim = torch.view_as_complex(buf[:m * C].view(-1, 2))
        ref = psi_ref[c0 * amps:(c0 + m) * amps]
        ov += complex(torch.sum(torch.conj(ref) * sim).item())
        n2 += float(torch.sum(sim.real * sim.real + sim.imag * sim.imag).item())
    return ov, n2
