"""GPU codec parity: streams from the HIP encoder equal the oracle's byte for
byte, and the HIP decoder rebuilds exactly the oracle's values."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import can be slow)

from oracle import qcz_oracle as oq
from tests.gpu_util import say, same_bits

pytestmark = pytest.mark.gpu


def families(rng, C):
    out = {
        "random": rng.normal(size=C) * 2.0 ** -12,
        "zeros": np.zeros(C),
        "const2": np.tile([0.125, -0.3], C // 2),
        "basis": np.r_[1.0, np.zeros(C - 1)],
        "wide": rng.normal(size=C) * np.ldexp(1.0, rng.integers(-900, 900, size=C)),
        "repeats": np.repeat(rng.normal(size=C // 8), 8),
        "same_binade": np.where(rng.random(C) < 0.5, -1, 1) * rng.uniform(1, 2, size=C) * 2.0 ** -15,
    }
    x = np.zeros(C)
    idx = rng.choice(C, size=max(1, C // 64), replace=False)
    x[idx] = rng.normal(size=idx.size)
    out["sparse"] = x
    x = rng.normal(size=C)
    x[1::2] = 0.0
    out["halfzero"] = x
    x = rng.normal(size=C)
    x[rng.random(C) < 0.3] = -0.0
    out["signed_zero"] = x
    x = rng.normal(size=C)
    x[5] = 2.0 ** -1070                       # subnormal: chunk stays lossless
    out["subnormal"] = x
    x = rng.normal(size=C)
    x[C - 3] = -(2.0 ** -1060)                # only the last wavefront of the chunk sees it
    out["subnormal_late"] = x
    x = np.zeros(C)
    x[-1] = -3.5
    out["last_only"] = x
    return out


@pytest.mark.parametrize("C", [128, 512, 2048])
def test_encode_matches_oracle_bytes(C):
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(C)
    fam = families(rng, C)
    names = sorted(fam)
    X = np.stack([fam[k] for k in names])
    for level in range(6):
        say("encode C=%d level=%d chunks=%d" % (C, level, len(names)))
        slots, sizes = qcz.encode_chunks(torch.from_numpy(X).cuda(), level)
        slots = slots.cpu().numpy()
        sizes = sizes.cpu().numpy()
        for i, k in enumerate(names):
            ref = oq.encode_chunk(X[i], level)
            got = slots[i, :sizes[i]].tobytes()
            assert got == ref, (k, level, len(got), len(ref))


@pytest.mark.parametrize("C", [128, 2048])
def test_decode_matches_oracle_values(C):
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(C + 1)
    fam = families(rng, C)
    names = sorted(fam)
    slot = (qcz.chunk_cap(C) + 3) & ~3
    for level in range(6):
        S = np.zeros((len(names), slot), dtype=np.uint8)
        sz = np.zeros(len(names), dtype=np.int32)
        refs = []
        for i, k in enumerate(names):
            b = oq.encode_chunk(fam[k], level)
            S[i, :len(b)] = np.frombuffer(b, dtype=np.uint8)
            sz[i] = len(b)
            refs.append(oq.decode_chunk(b, C))
        say("decode C=%d level=%d" % (C, level))
        out = qcz.decode_chunks(torch.from_numpy(S).cuda(), torch.from_numpy(sz).cuda(), C).cpu().numpy()
        for i, k in enumerate(names):
            assert same_bits(out[i], refs[i]), (k, level)


def test_encode_many_random_chunks():
    import torch
    from paper_1911_04034_amd import qcz
    rng = np.random.default_rng(77)
    C, n = 2048, 301                           # odd count: the last workgroup has one slot
    X = rng.normal(size=(n, C)) * 2.0 ** rng.integers(-30, 0, size=(n, 1))
    X[::7, ::3] = 0.0
    for level in (0, 2, 5):
        say("encode many level=%d" % level)
        slots, sizes = qcz.encode_chunks(torch.from_numpy(X).cuda(), level)
        slots, sizes = slots.cpu().numpy(), sizes.cpu().numpy()
        for i in range(0, n, 10):
            assert slots[i, :sizes[i]].tobytes() == oq.encode_chunk(X[i], level)
        dec = qcz.decode_chunks(torch.from_numpy(slots).cuda(), torch.from_numpy(sizes).cuda(), C).cpu().numpy()
        assert same_bits(dec, oq.truncate(X, level) if level else X)
