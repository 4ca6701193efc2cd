"""GPU parity of the per-block level selector: block statistics, per-level
sizes, the network's forward pass, gradient and Adam step, the per-block
fidelity ledger and the attached selector, against the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as mr
from oracle import qcz_oracle as oq
from oracle import select_ref as sr
from paper_1911_04034_amd import circuits as cc
from tests.gpu_util import assert_same_chunks, say

pytestmark = pytest.mark.gpu


def pair(n, bl, mode, level, gates, levels=None, **kw):
    from paper_1911_04034_amd import qcz
    g = qcz.State(n, bl, mode=mode, level=level, pool_bytes=64 << 20, **kw)
    o = oq.Sim(n, bl, mode, level)
    if levels is not None:
        g.set_block_levels(levels)
        for b, lv in enumerate(levels):
            o.set_block_level(b, int(lv))
    if len(gates):
        assert g.apply(gates) == len(gates)
        assert o.apply(gates) == len(gates)
    return g, o


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(scale=scale, size=mr.N_PARAMS)


@pytest.mark.parametrize("n,bl,level,seed", [(12, 8, 2, 1), (12, 11, 1, 2), (13, 10, 3, 3), (11, 6, 0, 4)])
def test_block_features_match_oracle(n, bl, level, seed):
    rng = np.random.default_rng(seed)
    nb = 1 << (n - bl)
    levels = rng.integers(0, 6, size=nb).astype(np.uint8)
    gates = cc.concat([cc.random_circuit_small(n, depth=6, seed=seed), cc.grover_prefix(n)[: n // 2]])
    say("features n=%d bl=%d" % (n, bl))
    g, o = pair(n, bl, oq.MODE_PERBLOCK, level, gates, levels)
    assert_same_chunks(g, o, "before statistics")
    for beta, mask in ((1e-4, 0), (0.0, nb - 1)):
        X, n2 = g.block_stats(beta, mask)
        F, n2o = sr.block_features(o, levels, beta, mask)
        Xg = X.cpu().numpy()
        assert np.allclose(n2.cpu().numpy(), n2o, rtol=1e-12, atol=1e-300)
        Fo = F.astype(np.float32)
        assert np.allclose(Xg[:, 0], Fo[:, 0], rtol=0, atol=2e-7)
        assert np.array_equal(Xg[:, 1:], Fo[:, 1:])


@pytest.mark.parametrize("n,bl,level", [(12, 8, 2), (13, 11, 0), (12, 10, 4)])
def test_level_sizes_match_oracle(n, bl, level):
    gates = cc.random_circuit_small(n, depth=8, seed=n + level)
    say("level sizes n=%d bl=%d level=%d" % (n, bl, level))
    g, o = pair(n, bl, oq.MODE_FIXED if level else oq.MODE_LOSSLESS, level, gates)
    S = g.block_level_sizes().cpu().numpy().astype(np.uint64)
    assert np.array_equal(S, sr.block_level_sizes(o))


@pytest.mark.parametrize("N", [1, 255, 1000])
def test_mlp_forward_matches_oracle(N):
    from paper_1911_04034_amd import qcz
    theta = _params(10 + N)
    X = np.random.default_rng(N).normal(size=(N, 16))
    say("mlp forward N=%d" % N)
    probs, lev = qcz.mlp_forward(torch.tensor(theta, dtype=torch.float32, device="cuda"),
                                 torch.tensor(X, dtype=torch.float32, device="cuda"))
    p_ref, _ = mr.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert np.allclose(probs.cpu().numpy(), p_ref, rtol=0, atol=2e-5)
    srt = np.sort(p_ref, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-4
    assert np.array_equal(lev.cpu().numpy()[clear], np.argmax(p_ref, axis=1)[clear])


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)


@pytest.mark.parametrize("N", [5, 777, 2100])
def test_mlp_gradient_matches_oracle(N):
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(100 + N)
    theta = _params(20 + N).astype(np.float32)
    X = rng.normal(size=(N, 16)).astype(np.float32)
    y = rng.integers(0, 6, size=N).astype(np.uint8)
    P = torch.tensor(theta, device="cuda")
    tr = qcz.MLPTrainer(P, N)
    say("mlp gradient N=%d" % N)
    loss = tr.step(torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda"), 0.0, update=False)
    L_ref, g_ref = mr.grad(theta.astype(np.float64), X.astype(np.float64), y)
    assert loss == pytest.approx(L_ref, rel=1e-5)
    g = tr.grad.cpu().numpy().astype(np.float64)
    for part, part_ref in zip(mr.unpack(g), mr.unpack(g_ref)):
        assert _rel(part, part_ref) < 1e-4
    assert np.array_equal(P.cpu().numpy(), theta)   # step 0 leaves the parameters alone


def test_adam_steps_match_oracle():
    from paper_1911_04034_amd import qcz
    N = 300
    rng = np.random.default_rng(7)
    theta = _params(7).astype(np.float32)
    X = rng.normal(size=(N, 16)).astype(np.float32)
    y = rng.integers(0, 6, size=N).astype(np.uint8)
    P = torch.tensor(theta, device="cuda")
    tr = qcz.MLPTrainer(P, N)
    Xd, yd = torch.tensor(X, device="cuda"), torch.tensor(y, device="cuda")
    m = np.zeros(mr.N_PARAMS)
    v = np.zeros(mr.N_PARAMS)
    lr = 1e-2
    for t in range(1, 4):
        before = P.cpu().numpy().astype(np.float64)
        say("adam step %d" % t)
        tr.step(Xd, yd, lr)
        _, g_ref = mr.grad(before, X.astype(np.float64), y)
        ref, m, v = mr.adam(before, m, v, g_ref, lr, t)
        after = P.cpu().numpy().astype(np.float64)
        big = np.abs(g_ref) > 1e-3 * np.max(np.abs(g_ref))
        assert np.max(np.abs(after - ref)[big]) < 1e-3 * lr


def test_perblock_ledger_matches_oracle():
    n, bl = 12, 8
    rng = np.random.default_rng(3)
    levels = rng.integers(0, 6, size=16).astype(np.uint8)
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 80, 3)])
    say("perblock ledger")
    g, o = pair(n, bl, oq.MODE_PERBLOCK, 0, gates, levels, batch=16)
    assert_same_chunks(g, o, "per-block levels")
    fg, fo = g.footprint(), o.footprint()
    assert fg["lossy_steps"] == fo["lossy_steps"]
    assert fg["fidelity_lower_bound"] == pytest.approx(fo["fidelity_lower_bound_weighted"], rel=1e-12)


def test_select_levels_projects_the_network_choice():
    from paper_1911_04034_amd import qcz
    n, bl = 13, 9
    gates = cc.concat([cc.grover_prefix(n), cc.random_circuit_small(n, depth=4, seed=5)])
    g, _ = pair(n, bl, oq.MODE_PERBLOCK, 2, gates)
    params = torch.tensor(_params(5, scale=1.0), dtype=torch.float32, device="cuda")
    for beta, mask in ((1e-5, 0), (1e-3, 0b1010), (1e-3, 0b1), (0.0, 0)):
        say("select beta=%g mask=%d" % (beta, mask))
        X, n2 = g.block_stats(beta, mask)
        _, lev = qcz.mlp_forward(params, X)
        w = n2.cpu().numpy()
        w = w / w.sum()
        want = sr.select_from_network(lev.cpu().numpy(), w, beta, mask)
        got = g.select_levels(params, beta, mask)
        assert np.array_equal(got, want)
        assert sr._weighted(got, w, mask) <= beta * sr.SLACK


def test_attached_selector_equals_manual_selection():
    from paper_1911_04034_amd import qcz
    n, bl, K, beta = 12, 8, 7, 1e-4
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 40, 9)])
    params = torch.tensor(_params(9, scale=1.0), dtype=torch.float32, device="cuda")
    a = qcz.State(n, bl, mode=qcz.MODE_PERBLOCK, level=0, pool_bytes=64 << 20, batch=5)
    b = qcz.State(n, bl, mode=qcz.MODE_PERBLOCK, level=0, pool_bytes=64 << 20, batch=64)
    a.set_selector(params, beta, K)
    say("attached selector")
    assert a.apply(gates) == len(gates)
    for k in range(0, len(gates), K):
        win = gates[k:k + K]
        mask = 0
        for gt in win:
            if gt["kind"] in (0, 3) and gt["target"] >= bl:
                mask |= 1 << (int(gt["target"]) - bl)
        b.select_levels(params, beta, mask)
        b.apply(win)
    for c in range(a.nchunks):
        assert a.export_chunk(c) == b.export_chunk(c)
    assert a.footprint()["fidelity_lower_bound"] == pytest.approx(b.footprint()["fidelity_lower_bound"], rel=1e-14)
