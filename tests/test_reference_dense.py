"""The uncompressed torch reference used for fidelity measurements agrees
with the oracle's dense simulator (which is pinned by Kronecker products)."""
import numpy as np
import torch

from oracle import qcz_oracle as oq
from paper_1911_04034_amd import circuits as cc
import dense_ref as ref


def test_reference_matches_oracle_dense_all_kinds():
    n = 8
    gates = cc.concat([cc.grover_prefix(n), cc.random_unitary_gates(n, 150, 3), cc.grid_rcs(2, 4, 4, 5),
                       cc.qaoa(8, 2, 3, 6)[0]])
    psi = ref.run(gates, n, ref.zero_state(n, device="cpu"))
    want = oq.apply_dense(np.eye(1, 1 << n, dtype=np.complex128)[0], n, gates)
    assert np.allclose(psi.numpy(), want, rtol=0, atol=1e-13)
    assert abs(torch.linalg.vector_norm(psi).item() - 1.0) < 1e-12
