"""Host-side selector logic of libqcz (no device work): Lagrangian labels and
budget projection equal the oracle's choices on the same inputs."""
import numpy as np
import pytest

from oracle import select_ref as sr
from paper_1911_04034_amd import qcz


def _instance(seed, B, ties=False):
    rng = np.random.default_rng(seed)
    S = np.sort(rng.integers(20, 9000, size=(B, 6)), axis=1)[:, ::-1].astype(np.uint64)
    if ties:
        S[::3, 2] = S[::3, 1]                    # levels with equal sizes
        S[1::4] = 20                             # blocks of two constants: flat size curve
    w = rng.random(B) ** 4
    w[1::7] = 0.0
    w /= w.sum()
    return S, w


@pytest.mark.parametrize("seed,B,beta,mask", [(0, 1, 1e-5, 0), (1, 4, 1e-4, 0b10), (2, 32, 1e-5, 0),
                                              (3, 64, 3e-3, 0b100001), (4, 256, 1e-2, 0b1111),
                                              (5, 128, 0.0, 0b1), (6, 64, 1.0, 0b111111), (7, 128, 2e-4, 0b1010000)])
@pytest.mark.parametrize("ties", [False, True])
def test_labels_equal_oracle(seed, B, beta, mask, ties):
    S, w = _instance(seed, B, ties)
    got = qcz.label_levels(S, w, beta, mask)
    assert np.array_equal(got, sr.label_levels(S, w, beta, mask))
    assert sr._weighted(got, w, mask) <= beta * sr.SLACK


def test_labels_uniform_weights_at_a_level_bound():
    """Uniform weights and beta = delta_l: the in-order sum of w * delta_l
    may round above beta; the slack keeps the uniform choice feasible."""
    B = 128
    S = np.tile(np.array([900, 500, 450, 400, 350, 300], dtype=np.uint64), (B, 1))
    w = np.full(B, 1.0 / B)
    for lev in range(1, 6):
        got = qcz.label_levels(S, w, sr.DELTA[lev])
        assert np.array_equal(got, sr.label_levels(S, w, sr.DELTA[lev]))
        assert np.all(got == lev)


@pytest.mark.parametrize("seed,B,beta,mask", [(0, 4, 1e-5, 0), (1, 32, 1e-4, 0b10001), (2, 256, 1e-3, 0),
                                              (3, 16, 0.0, 0b11), (4, 64, 0.5, 0b111111), (5, 128, 3e-5, 0b1000000)])
def test_projection_equals_oracle(seed, B, beta, mask):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, 6, size=B).astype(np.uint8)
    w = rng.random(B) ** 3
    w /= w.sum()
    got = qcz.project_levels(L, w, beta, mask)
    assert np.array_equal(got, sr.project_levels(L, w, beta, mask))
    assert np.all(got <= L)
    assert sr._weighted(got, w, mask) <= beta * sr.SLACK


def test_host_calls_reject_bad_input():
    with pytest.raises(qcz.QczError):
        qcz.label_levels(np.zeros((2, 6), np.uint64), np.array([0.5, -0.5]), 1e-5)
    with pytest.raises(qcz.QczError):
        qcz.project_levels([6, 0], np.array([0.5, 0.5]), 1e-5)
    with pytest.raises(qcz.QczError):
        qcz.project_levels([1, 0], np.array([0.5, 0.5]), -1.0)
    with pytest.raises(qcz.QczError):
        qcz.project_levels([1, 0], np.array([0.5, 0.5]), 1e-3, mask=0b10)   # bit beyond the block index
    with pytest.raises(qcz.QczError):
        qcz.label_levels(np.zeros((3, 6), np.uint64), np.full(3, 1 / 3), 1e-3)   # not a power of two
