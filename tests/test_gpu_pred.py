"""GPU parity of Solution B (Sec. 4.2: log-domain quantization, per-part
prediction, 16,384 symbols, Huffman codes; header mode 3): streams from the
HIP encoder equal the oracle's byte for byte, and the HIP decoder rebuilds
the oracle's values, also when Solution B and Solution C streams share one
decode call."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from tests.gpu_util import say, same_bits
from tests.test_gpu_codec import families

pytestmark = pytest.mark.gpu


def pred_families(rng, C):
    f = families(rng, C)
    f["smooth"] = np.repeat(np.cos(np.linspace(0, 3, C // 2)), 2) * 1e-3
    ph = rng.uniform(0, 2 * np.pi, size=C // 2)
    f["phases"] = np.stack([np.cos(ph), np.sin(ph)], axis=1).reshape(-1) * 2.0 ** -17
    sp = rng.normal(size=C)
    sp[3], sp[10], sp[11], sp[20], sp[21] = 5e-324, np.inf, -np.inf, 1.7976931348623157e308, -0.0
    sp[30] = np.nan
    f["specials"] = sp
    f["negzeros"] = -np.zeros(C)
    few = rng.choice([0.25, -0.25, 0.5, 1e-3], size=C)
    f["few_values"] = few
    return f


@pytest.mark.parametrize("C", [256, 512, 2048])
def test_pred_encode_matches_oracle_bytes(C):
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(1300 + C)
    fam = pred_families(rng, C)
    names = sorted(fam)
    X = np.stack([fam[k] for k in names])
    for level in range(1, 6):
        say("solution B encode C=%d level=%d chunks=%d" % (C, level, len(names)))
        slots, sizes = qcz.encode_chunks(torch.from_numpy(X).cuda(), level, codec_flags=qcz.CODEC_PREDICT)
        s_np, z_np = slots.cpu().numpy(), sizes.cpu().numpy()
        for i, k in enumerate(names):
            ref = oq.encode_pred(X[i], level)
            assert s_np[i, :z_np[i]].tobytes() == ref, (k, level, int(z_np[i]), len(ref))
        dec = qcz.decode_chunks(slots, sizes, C).cpu().numpy()
        for i, k in enumerate(names):
            assert same_bits(dec[i], oq.decode_chunk(oq.encode_pred(X[i], level), C)), (k, level)


def test_pred_many_chunks_and_mixed_decode():
    """301 chunks at every level; then one decode call over a mix of Solution
    B and Solution C streams (each kernel takes its own)."""
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(77)
    C, n = 2048, 301
    ph = rng.uniform(0, 2 * np.pi, size=(n, C // 2))
    X = np.stack([np.cos(ph), np.sin(ph)], axis=2).reshape(n, C) * 2.0 ** rng.integers(-30, 0, size=(n, 1))
    X[::5, ::3] = 0.0
    for level in range(1, 6):
        say("solution B many chunks level=%d" % level)
        slots, sizes = qcz.encode_chunks(torch.from_numpy(X).cuda(), level, codec_flags=qcz.CODEC_PREDICT)
        s_np, z_np = slots.cpu().numpy(), sizes.cpu().numpy()
        for i in range(0, n, 9):
            assert s_np[i, :z_np[i]].tobytes() == oq.encode_pred(X[i], level), (i, level)
    level = 2
    sb, zb = qcz.encode_chunks(torch.from_numpy(X).cuda(), level, codec_flags=qcz.CODEC_PREDICT)
    sc, zc = qcz.encode_chunks(torch.from_numpy(X).cuda(), level)
    slot = sb.shape[1]
    mix = torch.zeros_like(sb)
    mix[0::2] = sb[0::2]
    mix[1::2, :sc.shape[1]] = sc[1::2]
    zm = zb.clone()
    zm[1::2] = zc[1::2]
    say("mixed decode (slot %d)" % slot)
    dec = qcz.decode_chunks(mix, zm, C).cpu().numpy()
    for i in range(n):
        ref = oq.decode_chunk(oq.encode_pred(X[i], level) if i % 2 == 0 else oq.encode_chunk(X[i], level), C)
        assert same_bits(dec[i], ref), i


def test_pred_rejects_lossless_small_chunks_and_mixed_flags():
    import torch
    from paper_1911_04034_amd import qcz
    x = torch.zeros((2, 2048), dtype=torch.float64, device="cuda")
    with pytest.raises(qcz.QczError):
        qcz.encode_chunks(x, 0, codec_flags=qcz.CODEC_PREDICT)
    with pytest.raises(qcz.QczError):
        qcz.encode_chunks(torch.zeros((2, 128), dtype=torch.float64, device="cuda"), 1, codec_flags=qcz.CODEC_PREDICT)
    with pytest.raises(qcz.QczError):
        qcz.encode_chunks(x, 1, codec_flags=qcz.CODEC_PREDICT | qcz.CODEC_ENTROPY)
