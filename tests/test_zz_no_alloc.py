"""The no-allocation training step (qcz_mlp_train_step_noalloc) against the
workspace variant (qcz_mlp_train_step): same loss, gradient, Adam moments and
parameters, bit for bit (the same kernels in the same order), on two calls
in a row, the second with fewer samples than the first; sizes beyond the
static workspace are rejected before any work."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

QCZ_E_NOMEM = -2


def _inputs(n_samples, seed):
    g = torch.Generator().manual_seed(seed)
    X = torch.randn(n_samples, 16, generator=g, dtype=torch.float32)
    y = torch.randint(0, 6, (n_samples,), generator=g, dtype=torch.uint8)
    p = 0.1 * torch.randn(5638, generator=g, dtype=torch.float32)
    m = 0.01 * torch.randn(5638, generator=g, dtype=torch.float32)
    v = 0.01 * torch.rand(5638, generator=g, dtype=torch.float32)
    return [t.cuda() for t in (X, y, p, m, v)]


def _step(L, noalloc, X, y, p, m, v, step, stream):
    grad = torch.full((5638,), np.nan, dtype=torch.float32, device="cuda")
    loss = torch.full((1,), np.nan, dtype=torch.float32, device="cuda")
    n = X.shape[0]
    if noalloc:
        rc = L.qcz_mlp_train_step_noalloc(p.data_ptr(), m.data_ptr(), v.data_ptr(), X.data_ptr(), y.data_ptr(), n,
                                          ctypes.c_float(3e-3), step, grad.data_ptr(), loss.data_ptr(),
                                          stream.cuda_stream)
    else:
        work = torch.empty(L.qcz_mlp_workspace_bytes(n), dtype=torch.uint8, device="cuda")
        rc = L.qcz_mlp_train_step(p.data_ptr(), m.data_ptr(), v.data_ptr(), X.data_ptr(), y.data_ptr(), n,
                                  ctypes.c_float(3e-3), step, grad.data_ptr(), loss.data_ptr(), work.data_ptr(),
                                  work.numel(), stream.cuda_stream)
    stream.synchronize()
    return rc, grad.cpu().numpy(), loss.cpu().numpy()


def _bits(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def test_noalloc_train_step_equals_workspace_variant():
    from paper_1911_04034_amd import qcz
    L = qcz.load()
    stream = torch.cuda.Stream()
    for n_samples, seed, step in ((6000, 1, 1), (1500, 2, 3)):   # second call: a smaller input
        X, y, p, m, v = _inputs(n_samples, seed)
        ref = [t.clone() for t in (p, m, v)]
        rc_a, g_a, l_a = _step(L, False, X, y, ref[0], ref[1], ref[2], step, stream)
        rc_b, g_b, l_b = _step(L, True, X, y, p, m, v, step, stream)
        assert rc_a == 0 and rc_b == 0
        assert np.all(np.isfinite(g_b)) and np.isfinite(l_b[0])
        assert np.array_equal(_bits(g_a), _bits(g_b)) and np.array_equal(_bits(l_a), _bits(l_b))
        for a, b in zip(ref, (p, m, v)):
            assert np.array_equal(_bits(a.cpu().numpy()), _bits(b.cpu().numpy()))


def test_noalloc_train_step_rejects_more_samples_than_its_workspace():
    from paper_1911_04034_amd import qcz
    L = qcz.load()
    stream = torch.cuda.Stream()
    X, y, p, m, v = _inputs(8193, 3)
    before = p.clone()
    rc, g, loss = _step(L, True, X, y, p, m, v, 1, stream)
    assert rc == QCZ_E_NOMEM
    assert np.all(np.isnan(g)) and np.isnan(loss[0])   # nothing ran
    assert torch.equal(p, before)
