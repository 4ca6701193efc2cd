"""Pins of the oracle's gate arithmetic (Sec. 2.1 Eq. (5); Sec. 3.1 Eqs. (6),
(7)) against dense Kronecker matrices built here with numpy, and against the
closed forms of the Sec. 5.3 benchmarks (Grover, QFT)."""
import math

import numpy as np
import pytest

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc

I2 = np.eye(2, dtype=np.complex128)


def full_matrix(g, n):
    """Dense 2^n x 2^n operator of one gate record, from Eq. (5):
    A = I^(n-k-1) (x) U (x) I^(k), and projectors for controls."""
    kind = int(g["kind"][0])
    q, q2 = int(g["target"][0]), int(g["target2"][0])
    mask = int(g["control_mask"][0])
    m = g["m"][0]
    N = 1 << n
    idx = np.arange(N)
    ctrl_ok = (idx & mask) == mask
    if kind in (cc.U1, cc.X):
        U = (np.array([[m[0] + 1j * m[1], m[2] + 1j * m[3]], [m[4] + 1j * m[5], m[6] + 1j * m[7]]])
             if kind == cc.U1 else np.array([[0, 1], [1, 0]], dtype=np.complex128))
        A = np.array([[1.0 + 0j]])
        for k in range(n - 1, -1, -1):          # leftmost factor = highest qubit
            A = np.kron(A, U if k == q else I2)
        # controlled version: apply A only on the control-satisfied subspace
        P = np.diag(ctrl_ok.astype(np.complex128))
        return P @ A @ P + np.diag((~ctrl_ok).astype(np.complex128))
    if kind in (cc.DIAG1, cc.DIAG2):
        d = np.ones(N, dtype=np.complex128)
        for i in range(N):
            if not ctrl_ok[i]:
                continue
            j = ((i >> q) & 1) if kind == cc.DIAG1 else 2 * ((i >> q2) & 1) + ((i >> q) & 1)
            d[i] = m[2 * j] + 1j * m[2 * j + 1]
        return np.diag(d)
    if kind == cc.MCZ:
        return np.diag(np.where(ctrl_ok, -1.0, 1.0).astype(np.complex128))
    raise ValueError(kind)


@pytest.mark.parametrize("seed", range(6))
def test_gates_match_kronecker_matrices(seed):
    n = 5
    gates = cc.random_unitary_gates(n, 40, seed)
    psi = cc.random_state(n, seed + 50)
    ref = psi.copy()
    for k in range(len(gates)):
        ref = full_matrix(gates[k:k + 1], n) @ ref
    out = oq.apply_dense(psi, n, gates)
    assert np.max(np.abs(out - ref)) < 1e-13


def test_single_gate_kinds_exact_where_exact():
    n = 4
    psi = cc.random_state(n, 3)
    # X and MCZ are permutations / sign flips: bit exact
    out = oq.apply_dense(psi, n, cc.x(2, controls=(0,)))
    ref = psi.copy()
    for i in range(1 << n):
        if (i >> 0) & 1 and not (i >> 2) & 1:
            ref[i], ref[i | 4] = psi[i | 4], psi[i]
    assert np.array_equal(out, ref)
    out = oq.apply_dense(psi, n, cc.mcz((1, 3)))
    ref = psi.copy()
    for i in range(1 << n):
        if (i & 0b1010) == 0b1010:
            ref[i] = -psi[i]
    assert np.array_equal(out, ref)


def test_hadamard_all_from_zero():
    n = 8
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    out = oq.apply_dense(psi, n, cc.grover_prefix(n))
    assert np.allclose(out, 2.0 ** (-n / 2), rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,iters", [(6, 3), (8, 12), (9, 5)])
def test_grover_closed_form(n, iters):
    gates, w = cc.grover(n, iters, seed=n)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    out = oq.apply_dense(psi, n, gates)
    theta = math.asin(2.0 ** (-n / 2))
    sign = (-1) ** iters                      # each iteration is -G
    marked = sign * math.sin((2 * iters + 1) * theta)
    other = sign * math.cos((2 * iters + 1) * theta) / math.sqrt((1 << n) - 1)
    expect = np.full(1 << n, other, dtype=np.complex128)
    expect[w] = marked
    assert np.max(np.abs(out - expect)) < 1e-12


def bitrev(y, n):
    return int(format(y, "0%db" % n)[::-1], 2)


@pytest.mark.parametrize("n", [5, 8])
def test_qft_matches_fft(n):
    x_in = cc.qft_input(n, seed=n + 1)
    gates = cc.qft(n, x_in)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    out = oq.apply_dense(psi, n, gates)
    basis = np.zeros(1 << n, dtype=np.complex128)
    basis[x_in] = 1
    dft = np.fft.ifft(basis) * math.sqrt(1 << n)      # N^-1/2 sum_y e^{+2 pi i x y / N}
    expect = np.array([dft[bitrev(y, n)] for y in range(1 << n)])
    assert np.max(np.abs(out - expect)) < 1e-13


def inverse(gates):
    inv = gates[::-1].copy()
    for g in inv:
        m = g["m"]
        if g["kind"] == cc.U1:
            U = np.array([[m[0] + 1j * m[1], m[2] + 1j * m[3]], [m[4] + 1j * m[5], m[6] + 1j * m[7]]])
            Ui = U.conj().T
            g["m"][:] = [Ui[0, 0].real, Ui[0, 0].imag, Ui[0, 1].real, Ui[0, 1].imag,
                         Ui[1, 0].real, Ui[1, 0].imag, Ui[1, 1].real, Ui[1, 1].imag]
        elif g["kind"] in (cc.DIAG1, cc.DIAG2):
            g["m"][1::2] = -g["m"][1::2]
    return inv


def test_circuit_then_inverse_is_identity_and_norm_kept():
    n = 10
    gates = cc.random_circuit_small(n, depth=8, seed=9)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1
    mid = oq.apply_dense(psi, n, gates)
    assert abs(np.linalg.norm(mid) - 1) < 1e-12
    back = oq.apply_dense(mid, n, inverse(gates))
    assert np.max(np.abs(back - psi)) < 1e-12


def test_gate_check_rejects_malformed():
    n = 4
    assert oq.gate_check(cc.h(3), n)
    assert not oq.gate_check(cc.h(4), n)                       # qubit out of range
    assert not oq.gate_check(cc.x(1, controls=(1,)), n)        # target is a control
    g = cc.h(0)
    g["m"][0, 0] = np.nan
    assert not oq.gate_check(g, n)                             # non-finite matrix
    assert not oq.gate_check(cc.diag2(1, 1, [1, 1, 1, 1]), n)  # same qubit twice
