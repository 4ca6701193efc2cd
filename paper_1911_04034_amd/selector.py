"""Training and evaluation of the per-block level selector.

Sec. 3.7 relaxes one error bound for the whole state; the selector picks one
bound per block for each window of `period` gates (the C ABI of
include/qcz.h holds every computation; this module strings the calls
together):

* teacher labels: for the state at the start of a window, the window is run
  on a copy of the state at each of the six uniform levels and the padded
  bytes of every block at the window's end are read back; qcz_label_levels
  then picks per block the level that minimises those bytes under the
  window's budget sum_c W_c delta(max level in coset c) <= beta (cosets of the
  block-index bits the window's gates flip, so the budget holds at every
  gate of the window);
* training: block features (qcz_block_stats) and the teacher labels of
  traced runs, full-batch cross-entropy with Adam on the device
  (qcz_mlp_train_step);
* use: qcz_set_selector attaches the trained parameters; every `period`
  gates the state re-selects its block levels (features -> network -> at
  least the rule's level -> budget projection).

Inputs are synthetic circuits from ``circuits``.
"""
from __future__ import annotations

import math

import numpy as np

from . import qcz

DELTA = [0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1]


def _torch():
    import torch
    return torch


def level_of(beta: float) -> int:
    return DELTA.index(beta)


def block_bytes(state) -> np.ndarray:
    """Padded stream bytes of every block of a state (host int64)."""
    sizes = state.chunk_sizes().astype(np.int64)
    nb = 1 << (state.n - state.block_log2)
    return ((sizes + 3) & ~3).reshape(nb, -1).sum(axis=1)


def future_sizes(state, scratch, window) -> np.ndarray:
    """Bytes of every block at the end of `window` when the whole window runs
    at each uniform level, starting from `state` (uint64 [nblocks, 6])."""
    nb = 1 << (state.n - state.block_log2)
    S = np.zeros((nb, 6), dtype=np.uint64)
    for lev in range(6):
        scratch.copy_from(state)
        scratch.set_block_levels(np.full(nb, lev, dtype=np.uint8))
        scratch.apply(window)
        S[:, lev] = block_bytes(scratch).astype(np.uint64)
    return S


def teacher_trace(gates, n: int, block_log2: int, beta: float, period: int, pool_bytes: int | None = None):
    """Run `gates` in windows of `period` with the teacher's block levels.
    Returns (features cuda float32 [N, 16], labels cuda uint8 [N], bytes
    after each window, fidelity lower bound)."""
    torch = _torch()
    st = qcz.State(n, block_log2, mode=qcz.MODE_PERBLOCK, level=0, pool_bytes=pool_bytes)
    scratch = qcz.State(n, block_log2, mode=qcz.MODE_PERBLOCK, level=0, pool_bytes=pool_bytes, stream=st.stream)
    Xs, ys, trace = [], [], []
    for k in range(0, len(gates), period):
        win = gates[k:k + period]
        mask = st.mixing_mask(win)
        X, n2 = st.block_stats(beta, mask)
        w = n2.cpu().numpy()
        w = w / w.sum()
        y = qcz.label_levels(future_sizes(st, scratch, win), w, beta, mask)
        Xs.append(X)
        ys.append(torch.from_numpy(y).to("cuda"))
        st.set_block_levels(y)
        st.apply(win)
        trace.append(st.footprint()["compressed_bytes"])
    return torch.cat(Xs), torch.cat(ys), np.array(trace), st.footprint()["fidelity_lower_bound"]


def init_params(seed: int = 0):
    """He-normal weights, zero biases (seeded), as a cuda float32 tensor."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 16), (64, 64), (6, 64)):
        parts.append(rng.normal(scale=math.sqrt(2.0 / cols), size=rows * cols))
        parts.append(np.zeros(rows))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == qcz.MLP_PARAMS
    return torch.tensor(theta, device="cuda")


def train(X, y, steps: int = 1500, lr: float = 3e-3, seed: int = 0):
    """Full-batch training on the device; returns (params, loss history)."""
    params = init_params(seed)
    tr = qcz.MLPTrainer(params, X.shape[0])
    losses = []
    for t in range(steps):
        sync = (t + 1) % 100 == 0 or t + 1 == steps
        loss = tr.step(X, y, lr, sync=sync)
        if sync:
            losses.append(loss)
    return params, losses


def accuracy(params, X, y) -> float:
    _, lev = qcz.mlp_forward(params, X)
    return float((lev == y).float().mean().item())


def run_rule(gates, n: int, block_log2: int, beta: float, period: int, pool_bytes: int | None = None):
    """The fixed-bound rule at beta: (bytes after each window, F_lb)."""
    st = qcz.State(n, block_log2, mode=qcz.MODE_FIXED, level=level_of(beta), pool_bytes=pool_bytes)
    trace = []
    for k in range(0, len(gates), period):
        st.apply(gates[k:k + period])
        trace.append(st.footprint()["compressed_bytes"])
    return np.array(trace), st.footprint()["fidelity_lower_bound"]


def run_selector(gates, n: int, block_log2: int, beta: float, period: int, params, pool_bytes: int | None = None):
    """The attached selector at budget beta: (bytes after each window, F_lb)."""
    st = qcz.State(n, block_log2, mode=qcz.MODE_PERBLOCK, level=0, pool_bytes=pool_bytes)
    st.set_selector(params, beta, period)
    trace = []
    for k in range(0, len(gates), period):
        st.apply(gates[k:k + period])
        trace.append(st.footprint()["compressed_bytes"])
    return np.array(trace), st.footprint()["fidelity_lower_bound"]


def training_set(circuits, betas, period: int):
    """Teacher traces of (gates, n, block_log2) circuits at each beta."""
    torch = _torch()
    Xs, ys = [], []
    for beta in betas:
        for gates, n, bl in circuits:
            X, y, _, _ = teacher_trace(gates, n, bl, beta, period)
            Xs.append(X)
            ys.append(y)
    return torch.cat(Xs), torch.cat(ys)
