"""Pins of the selector's references (oracle/mlp_ref.py, oracle/select_ref.py)
and of the per-block fidelity ledger: closed forms, central differences,
brute force on tiny instances and hand-worked examples."""
import itertools
import math

import numpy as np
import pytest

from oracle import mlp_ref as mr
from oracle import qcz_oracle as oq
from oracle import select_ref as sr
from paper_1911_04034_amd import circuits as cc


# ---------------------------------------------------------------- network --
def test_mlp_zero_parameters_closed_form():
    X = np.random.default_rng(0).normal(size=(9, 16))
    y = np.array([0, 1, 2, 3, 4, 5, 5, 5, 0])
    theta = np.zeros(mr.N_PARAMS)
    p, _ = mr.forward(theta, X)
    assert np.allclose(p, 1.0 / 6.0, rtol=0, atol=1e-15)
    L, g = mr.grad(theta, X, y)
    assert abs(L - math.log(6.0)) < 1e-14
    parts = mr.unpack(g)
    freq = np.bincount(y, minlength=6) / len(y)
    assert np.allclose(parts[5], 1.0 / 6.0 - freq, atol=1e-15)   # b3
    for k in range(5):
        assert not np.any(parts[k])   # every hidden unit is at ReLU'(0) = 0


def test_mlp_wiring_hand_network():
    """z_c = c * relu(a) through unit 0 of both hidden layers."""
    W1, b1, W2, b2, W3, b3 = [np.zeros(s) for s in mr.SHAPES]
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0
    W3[:, 0] = np.arange(6.0)
    theta = mr.pack([W1, b1, W2, b2, W3, b3])
    X = np.zeros((2, 16))
    X[0, 0] = 1.0
    X[1, 0] = -1.0
    p, _ = mr.forward(theta, X)
    e = np.exp(np.arange(6.0))
    assert np.allclose(p[0], e / e.sum(), rtol=1e-14)
    assert np.allclose(p[1], 1.0 / 6.0, rtol=1e-14)
    assert list(mr.predict(theta, X)) == [5, 0]


def test_mlp_gradient_central_differences():
    rng = np.random.default_rng(1)
    theta = rng.normal(scale=0.3, size=mr.N_PARAMS)
    X = rng.normal(size=(13, 16))
    y = rng.integers(0, 6, size=13)
    L, g = mr.grad(theta, X, y)
    assert abs(L - mr.loss(theta, X, y)) < 1e-14
    idx = np.concatenate([rng.choice(mr.N_PARAMS, size=300, replace=False),
                          np.arange(1024, 1088), np.arange(5632, 5638)])
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mr.loss(tp, X, y) - mr.loss(tm, X, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(g[k]), k


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, m, v = mr.adam(theta, np.zeros(50), np.zeros(50), g, 0.01, 1)
    assert np.allclose(t1, theta - 0.01 * g / (np.abs(g) + mr.EPS), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# --------------------------------------------------------- labels / budget --
def _tiny(seed, B):
    rng = np.random.default_rng(seed)
    S = np.sort(rng.integers(100, 4000, size=(B, 6)), axis=1)[:, ::-1].astype(np.uint64)
    w = rng.random(B)
    w /= w.sum()
    return S, w


def _cost(S, L):
    return int(sum(int(S[b, L[b]]) for b in range(len(L))))


@pytest.mark.parametrize("seed", range(6))
def test_labels_are_optimal_for_their_own_budget(seed):
    """A Lagrangian choice is the cheapest among all choices that use no more
    of the budget than it does (brute force over 6^4 choices)."""
    S, w = _tiny(seed, 4)
    beta = [1e-5, 3e-5, 1e-4, 2e-3, 0.02, 0.05][seed]
    L = sr.label_levels(S, w, beta)
    used = sr._weighted(L, w)
    assert used <= beta * sr.SLACK
    best = min(_cost(S, c) for c in itertools.product(range(6), repeat=4) if sr._weighted(c, w) <= used)
    assert _cost(S, L) == best


def test_labels_extremes():
    S, w = _tiny(7, 5)
    assert list(sr.label_levels(S, w, 1.0)) == [5] * 5          # budget never binds: smallest streams
    assert list(sr.label_levels(S, w, 0.0)) == [0] * 5          # no error allowed: lossless
    w0 = w.copy()
    w0[2] = 0.0                                                 # a block without weight costs nothing
    assert sr.label_levels(S, w0, 0.0)[2] == 5


@pytest.mark.parametrize("seed,mask", [(0, 0b01), (1, 0b10), (2, 0b11), (3, 0b101)])
def test_coset_labels_are_optimal_for_their_own_budget(seed, mask):
    """With a mixing mask the budget counts each coset's weight at its
    loosest level; brute force over 6^B choices."""
    B = 8 if mask == 0b101 else 4
    S, w = _tiny(10 + seed, B)
    beta = [1e-4, 2e-5, 3e-3, 1e-2][seed]
    L = sr.label_levels(S, w, beta, mask)
    used = sr._weighted(L, w, mask)
    assert used <= beta * sr.SLACK
    if B == 4:
        best = min(_cost(S, c) for c in itertools.product(range(6), repeat=B) if sr._weighted(c, w, mask) <= used)
        assert _cost(S, L) == best


def test_coset_weights_and_budget_hand_example():
    w = np.array([0.4, 0.1, 0.3, 0.2])
    ids, order, W = sr.coset_weights(w, 0b01)
    assert order == [0, 2] and W[0] == 0.5 and abs(W[2] - 0.5) < 1e-16
    # coset {0,1} at max level 3 (1e-3), coset {2,3} at max level 1 (1e-5)
    assert abs(sr._weighted([3, 0, 1, 1], w, 0b01) - (0.5 * 1e-3 + 0.5 * 1e-5)) < 1e-18
    # full mixing: one coset, the loosest block sets the bound for all the weight
    assert abs(sr._weighted([0, 0, 5, 0], w, 0b11) - 0.1) < 1e-16
    assert list(sr.project_levels([5, 0, 2, 5], w, 1e-2, 0b11)) == [4, 0, 2, 4]
    assert list(sr.project_levels([5, 0, 2, 5], w, 1e-3, 0b11)) == [3, 0, 2, 3]


def test_projection_hand_example():
    w = np.array([0.5, 0.3, 0.2])
    assert list(sr.project_levels([5, 5, 5], w, 0.01)) == [4, 4, 4]
    assert list(sr.project_levels([5, 1, 0], w, 1.0)) == [5, 1, 0]


def test_rule_level_and_floor_hand_example():
    # the loosest level with delta <= beta
    assert [sr.rule_level(b) for b in (0.0, 1e-6, 1e-5, 5e-5, 1e-4, 1e-3, 0.05, 1.0)] == [0, 0, 1, 1, 2, 3, 4, 5]
    w = np.array([0.5, 0.3, 0.2])
    # tighter choices are raised to the rule's level (here level 2 for 1e-4) ...
    assert list(sr.select_from_network([0, 1, 4], w, 1e-4)) == [2, 2, 2]
    # ... then the projection: [3, 5, 3] costs 0.98e-3 + 0.01 * 0.1 + 0.01e-3 > 1e-3; block 1
    # (largest W * delta) drops to 4, still over; block 0 drops to 2: 0.98e-4 + 1e-4 + 1e-5
    w = np.array([0.98, 0.01, 0.01])
    assert list(sr.select_from_network([0, 5, 3], w, 1e-3)) == [2, 4, 3]


@pytest.mark.parametrize("seed", range(6))
def test_floored_selection_meets_budget_and_rule(seed):
    """Random instances: the floored projection meets the coset budget, and
    a block below the rule's level only appears in a coset the projection
    had to lower (its loosest block is then at most the rule's level)."""
    rng = np.random.default_rng(seed)
    nb = 16
    w = rng.dirichlet(np.full(nb, 0.3))
    beta = float(rng.choice([1e-5, 1e-4, 1e-3]))
    mask = int(rng.integers(0, nb))
    lev = rng.integers(0, 6, size=nb)
    got = sr.select_from_network(lev, w, beta, mask)
    assert sr._weighted(got, w, mask) <= beta * sr.SLACK
    rule = sr.rule_level(beta)
    ids, order, W = sr.coset_weights(w, mask)
    for b in range(nb):
        if got[b] < rule:
            top = max(int(got[x]) for x in range(nb) if ids[x] == ids[b])
            assert top <= rule


# --------------------------------------------------------------- features --
def test_features_of_basis_state():
    n, bl = 12, 10
    s = oq.Sim(n, bl)
    F, n2 = sr.block_features(s, [0] * 4, 1e-5)
    M = 2 << bl
    assert n2[0] == 1.0 and not np.any(n2[1:])
    f = F[0]
    assert f[0] == math.log2(4) / 64
    assert f[1] == 1 - 1 / M and f[2] == 0 and f[3] == 0 and f[11] == 0
    assert f[4] == f[5] == f[6] == (M - 2) / M and f[7] == 0
    assert f[8] == 0.0
    for f in F[1:]:
        assert f[0] == -60 / 64 and f[1] == 1 and f[11] == -17
        assert f[4] == f[5] == f[6] == 1 and f[7] == 0 and f[8] == 1
        assert f[9] == 20 / (16 * 1024)
    assert np.allclose(F[:, 12], -1.0, rtol=1e-15) and np.all(F[:, 14] == 2 / 16) and np.all(F[:, 15] == 0)
    F2, _ = sr.block_features(s, [0] * 4, 1e-5, mask=0b11)
    assert np.all(F2[:, 15] == 2 / 16) and np.array_equal(F2[:, :15], F[:, :15])


def test_features_of_uniform_state():
    n, bl = 11, 9
    s = oq.Sim(n, bl)
    s.apply(cc.concat([cc.h(q) for q in range(n)]))
    F, n2 = sr.block_features(s, [0] * 4, 1e-3)
    assert np.allclose(n2, 0.25, rtol=1e-12)
    assert np.allclose(F[:, 0], 0.0, atol=1e-12)
    assert np.all(F[:, 1] == 0.5) and np.all(F[:, 3] == 0) and np.all(F[:, 8] == 1)
    assert np.all(F[:, 4] == 0) and np.all(F[:, 7] == 0)


# ------------------------------------------------------------ level sizes --
def test_level_sizes_properties():
    n, bl = 12, 10
    s = oq.Sim(n, bl)
    s.apply(cc.random_circuit_small(n, depth=8, seed=4))
    S = sr.block_level_sizes(s)
    # re-encoding at the current level reproduces the stored streams (idempotent truncation)
    cur = [sum((len(s.chunk(c)) + 3) & ~3 for c in range(b, b + 1)) for b in range(4)]
    assert list(S[:, 0]) == cur
    # a looser bound never needs more bytes
    assert np.all(np.diff(S.astype(np.int64), axis=1) <= 0)
    z = oq.Sim(n, bl)
    Sz = sr.block_level_sizes(z)
    assert np.all(Sz[1:] == 20)


# --------------------------------------------------- per-block fidelity --
def test_perblock_ledger_single_gate_closed_form():
    for lev in range(6):
        s = oq.Sim(10, 8, oq.MODE_PERBLOCK, lev)
        s.apply(cc.h(0))
        fp = s.footprint()
        n2 = float(np.sum(np.abs(np.array([1, 1]) / math.sqrt(2)) ** 2))
        assert abs(fp["fidelity_lower_bound_weighted"] - (1 - sr.DELTA[lev] * n2)) < 1e-15


def test_perblock_ledger_bounds_the_fidelity():
    """Uniform per-block level: same bytes as the fixed level, a ledger no
    lower than Eq. (11) (each step deducts delta times the touched share of
    the norm), and below the fidelity measured against the exact state."""
    n, bl, lev = 10, 6, 3
    gates = cc.random_circuit_small(n, depth=12, seed=8)
    a = oq.Sim(n, bl, oq.MODE_FIXED, lev)
    b = oq.Sim(n, bl, oq.MODE_PERBLOCK, lev)
    a.apply(gates)
    b.apply(gates)
    assert all(a.chunk(c) == b.chunk(c) for c in range(a.nchunks))
    fa, fb = a.footprint(), b.footprint()
    ideal = oq.apply_dense(np.eye(1, 1 << n, dtype=np.complex128)[0], n, gates)
    psi = b.state()
    f_norm = abs(np.vdot(ideal, psi)) / np.linalg.norm(psi)
    assert fb["fidelity_lower_bound_weighted"] <= f_norm
    assert fb["fidelity_lower_bound_weighted"] >= fa["fidelity_lower_bound"] - 1e-12
    z = oq.Sim(n, bl, oq.MODE_PERBLOCK, 0)
    z.apply(gates)
    assert z.footprint()["fidelity_lower_bound_weighted"] == 1.0


def test_perblock_ledger_counts_only_touched_chunks():
    """A gate controlled by a chunk-index qubit leaves half the chunks alone;
    only the touched half's norm enters the ledger."""
    n, bl, lev = 10, 6, 2
    s = oq.Sim(n, bl, oq.MODE_PERBLOCK, lev)
    s.apply(cc.concat([cc.h(q) for q in range(n)]))
    f0 = s.footprint()["fidelity_lower_bound_weighted"]
    g = cc.u1(0, np.array([[0, 1], [1, 0]], dtype=complex) * 1j, controls=[9])
    s.apply(g)
    f1 = s.footprint()["fidelity_lower_bound_weighted"]
    ratio = f1 / f0
    assert abs((1 - ratio) - sr.DELTA[lev] * 0.5) < 1e-12
