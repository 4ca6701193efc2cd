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
