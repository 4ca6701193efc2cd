"""Pins of the readout reference (oracle/readout_ref.py): the published
SplitMix64 outputs, basis states, exact inverse-CDF picks on a small
state, sampling frequencies, and the overlap's closed forms."""
import json
import math
import os

import numpy as np
import pytest

from oracle import readout_ref as rr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")


def test_splitmix64_published_outputs():
    for case in json.load(open(GOLDEN))["cases"]:
        for k, want in enumerate(case["outputs"]):
            assert rr.splitmix64(case["seed"], k) == int(want, 0)


def test_basis_state_always_sampled():
    psi = np.zeros(1 << 9, dtype=np.complex128)
    psi[300] = -1j
    assert np.all(rr.sample(psi, 128, 5, 200) == 300)


def test_inverse_cdf_picks_on_a_small_state():
    # |a|^2 = 0.1, 0.2, 0.3, 0.4 over four amplitudes in two chunks of two
    psi = np.sqrt(np.array([0.1, 0.2, 0.3, 0.4])).astype(np.complex128)
    got = rr.sample(psi, 2, 11, 64)
    for k in range(64):
        u = (rr.splitmix64(11, k) >> 11) * 2.0 ** -53
        want = int(np.searchsorted(np.cumsum([0.1, 0.2, 0.3, 0.4]), u * 1.0, side="right"))
        assert got[k] == min(want, 3)


def test_sampling_frequencies():
    rng = np.random.default_rng(3)
    psi = rng.normal(size=64) + 1j * rng.normal(size=64)
    psi[rng.random(64) < 0.3] = 0
    p = np.abs(psi) ** 2
    p /= p.sum()
    shots = 40000
    counts = np.bincount(rr.sample(psi, 16, 77, shots).astype(np.int64), minlength=64)
    assert np.all(counts[p == 0] == 0)
    expect = p * shots
    chi2 = np.sum((counts[p > 0] - expect[p > 0]) ** 2 / expect[p > 0])
    dof = int(np.sum(p > 0)) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_overlap_closed_forms():
    a = np.array([1, 1j, 0, -1]) / math.sqrt(3)
    assert rr.overlap(a, a) == pytest.approx(1.0)
    assert rr.overlap(a, 1j * a) == pytest.approx(1j)
    b = np.array([0, 0, 1, 0])
    assert rr.overlap(a, b) == 0


def test_sampler_agrees_with_the_plain_global_inverse_cdf():
    # The plain definition: index i with probability |a_i|^2 / sum |a|^2, drawn
    # by inverting the running sum over the whole vector in index order.  The
    # chunk-then-amplitude walk is the same inverse in exact arithmetic; only
    # draws within rounding distance of a boundary may differ.
    rng = np.random.default_rng(7)
    n, apc, shots, seed = 12, 64, 4000, 99
    psi = (rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)) * (rng.random(1 << n) < 0.7)
    psi /= np.linalg.norm(psi)
    got = rr.sample(psi, apc, seed, shots)
    p = np.abs(psi) ** 2
    cdf = np.cumsum(p)
    u = np.array([(rr.splitmix64(seed, k) >> 11) * 2.0 ** -53 for k in range(shots)])
    plain = np.minimum(np.searchsorted(cdf, u * cdf[-1], side="right"), (1 << n) - 1)
    assert np.mean(got == plain) >= 0.999
    assert np.all(p[got] > 0)
