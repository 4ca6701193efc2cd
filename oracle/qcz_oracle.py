"""ctypes front end of the CPU oracle (``qcz_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  It holds
no simulation arithmetic of its own beyond marshalling; everything that
decides a value happens in the C file, written from the paper:

* truncation to Sig_Bit_Count bits and the XOR leading-byte code
  (Sec. 4.2, Solution C, Eq. (12));
* the blockwise decompress -> update -> recompress loop (Sec. 3.1, 3.3);
* the variable error bound (Sec. 3.7) and the fidelity ledger (Sec. 3.8).

The fp64 reference of the learned level selector lives in ``mlp_ref.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qcz_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

N_LEVELS = 6
MODE_LOSSLESS, MODE_FIXED, MODE_ADAPTIVE, MODE_PERBLOCK = 0, 1, 2, 3
GATE_BYTES = 88


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction of a*b+c into an FMA)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        u8p = ctypes.POINTER(ctypes.c_uint8)
        dp = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        vp = ctypes.c_void_p
        L.oq_level_delta.restype = ctypes.c_double
        L.oq_level_delta.argtypes = [ctypes.c_int]
        L.oq_exp_of.restype = ctypes.c_int
        L.oq_exp_of.argtypes = [ctypes.c_double]
        L.oq_sig_bits.restype = ctypes.c_int
        L.oq_sig_bits.argtypes = [ctypes.c_int]
        L.oq_truncate_bits.restype = ctypes.c_uint64
        L.oq_truncate_bits.argtypes = [ctypes.c_uint64, ctypes.c_int]
        L.oq_truncate.restype = ctypes.c_double
        L.oq_truncate.argtypes = [ctypes.c_double, ctypes.c_int]
        L.oq_chunk_cap.restype = ctypes.c_size_t
        L.oq_chunk_cap.argtypes = [ctypes.c_int]
        L.oq_encode_chunk.restype = ctypes.c_size_t
        L.oq_encode_chunk.argtypes = [dp, ctypes.c_int, ctypes.c_int, u8p]
        L.oq_encode_chunk_ex.restype = ctypes.c_size_t
        L.oq_encode_chunk_ex.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p]
        L.oq_chunk_cap_forced.restype = ctypes.c_size_t
        L.oq_chunk_cap_forced.argtypes = [ctypes.c_int]
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oq_huff_lengths.restype = ctypes.c_int
        L.oq_huff_lengths.argtypes = [u32p, ctypes.c_int, u8p]
        L.oq_canon_codes.restype = ctypes.c_int
        L.oq_canon_codes.argtypes = [u8p, ctypes.c_int, u32p]
        L.oq_gate_job_ex.restype = ctypes.c_int
        L.oq_gate_job_ex.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint64, u8p, ctypes.c_size_t, ctypes.c_int, u8p,
                                     ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.c_uint64, u8p, ctypes.c_size_t, ctypes.c_int, u8p,
                                     ctypes.POINTER(ctypes.c_size_t)]
        L.oq_encode_pred.restype = ctypes.c_size_t
        L.oq_encode_pred.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
        L.oq_pred_cap.restype = ctypes.c_size_t
        L.oq_pred_cap.argtypes = [ctypes.c_int]
        L.oq_pred_symbols.restype = ctypes.c_int
        L.oq_pred_symbols.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
        L.oq_pred_huff_lengths.restype = ctypes.c_int
        L.oq_pred_huff_lengths.argtypes = [vp, ctypes.c_int, vp]
        L.oq_pred_width.restype = ctypes.c_int
        L.oq_pred_width.argtypes = [ctypes.c_int]
        L.oq_sim_set_codec.restype = None
        L.oq_sim_set_codec.argtypes = [vp, ctypes.c_int]
        L.oq_decode_chunk.restype = ctypes.c_int
        L.oq_decode_chunk.argtypes = [u8p, ctypes.c_size_t, ctypes.c_int, dp]
        L.oq_gate_size.restype = ctypes.c_size_t
        L.oq_gate_check.restype = ctypes.c_int
        L.oq_gate_check.argtypes = [vp, ctypes.c_int]
        L.oq_apply_gate_dense.restype = ctypes.c_int
        L.oq_apply_gate_dense.argtypes = [dp, ctypes.c_int, vp]
        L.oq_chunk_role.restype = ctypes.c_int
        L.oq_chunk_role.argtypes = [vp, ctypes.c_int, ctypes.c_uint64]
        L.oq_gate_job.restype = ctypes.c_int
        L.oq_gate_job.argtypes = [vp, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_uint64, u8p, ctypes.c_size_t, ctypes.c_int, u8p,
                                  ctypes.POINTER(ctypes.c_size_t),
                                  ctypes.c_uint64, u8p, ctypes.c_size_t, ctypes.c_int, u8p,
                                  ctypes.POINTER(ctypes.c_size_t)]
        L.oq_sim_create.restype = vp
        L.oq_sim_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
        L.oq_sim_destroy.argtypes = [vp]
        L.oq_sim_apply.restype = ctypes.c_long
        L.oq_sim_apply.argtypes = [vp, vp, ctypes.c_size_t]
        L.oq_sim_read_all.restype = ctypes.c_int
        L.oq_sim_read_all.argtypes = [vp, dp]
        L.oq_sim_chunk.restype = ctypes.c_size_t
        L.oq_sim_chunk.argtypes = [vp, ctypes.c_uint64, u8p, ctypes.c_size_t]
        L.oq_sim_set_chunk.restype = ctypes.c_int
        L.oq_sim_set_chunk.argtypes = [vp, ctypes.c_uint64, u8p, ctypes.c_size_t]
        L.oq_sim_set_block_level.restype = ctypes.c_int
        L.oq_sim_set_block_level.argtypes = [vp, ctypes.c_uint64, ctypes.c_int]
        L.oq_sim_footprint.argtypes = [vp, u64p, dp]
        L.oq_sim_compressed_bytes.restype = ctypes.c_uint64
        L.oq_sim_compressed_bytes.argtypes = [vp]
        L.oq_sim_chunk_log2.restype = ctypes.c_int
        L.oq_sim_chunk_log2.argtypes = [vp]
        assert L.oq_gate_size() == GATE_BYTES
        _lib = L
    return _lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _gates(g):
    g = np.ascontiguousarray(g)
    assert g.dtype.itemsize == GATE_BYTES, "gate records must be 88-byte structs"
    return g


# --------------------------------------------------------------------------
# scalar helpers (Eq. (12))
# --------------------------------------------------------------------------
def level_delta(level: int) -> float:
    return lib().oq_level_delta(level)


def exp_of(eps: float) -> int:
    return lib().oq_exp_of(eps)


def sig_bits(level: int) -> int:
    return lib().oq_sig_bits(level)


def truncate_bits(bits: int, K: int) -> int:
    return lib().oq_truncate_bits(bits, K)


def truncate(x, level: int):
    """Elementwise truncation of float64 values to the level's significant bits."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.empty_like(a)
    f = lib().oq_truncate
    flat_in, flat_out = a.reshape(-1), out.reshape(-1)
    for i in range(flat_in.size):
        flat_out[i] = f(float(flat_in[i]), level)
    return out


# --------------------------------------------------------------------------
# chunk codec
# --------------------------------------------------------------------------
def chunk_cap(C: int) -> int:
    return lib().oq_chunk_cap(C)


ENC_ENTROPY = 1     # the encoder may take the entropy-coded body
ENC_FORCE_ENT = 2   # test hook: always entropy-code the PACK / SPARSE body
ENC_FORCE_CODED = 4 # test hook: every lane with two or more symbols CODED, one symbol CONST
ENC_RESHUFFLE = 8   # Solution D: PACK / SPARSE values stored re parts first, then im parts (header bit 6)


def encode_chunk(x, level: int, flags: int = 0) -> bytes:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    C = x.size
    cap = lib().oq_chunk_cap_forced(C) if flags & ENC_FORCE_ENT else chunk_cap(C)
    buf = np.zeros(cap, dtype=np.uint8)
    n = lib().oq_encode_chunk_ex(_dp(x), C, level, flags, _u8(buf))
    if n == 0:
        raise ValueError("bad chunk size or level")
    return buf[:n].tobytes()


def encode_pred(x, level: int) -> bytes:
    """Solution B (Sec. 4.2): log-domain quantization, per-part prediction,
    16,384 bins, Huffman codes; lossy levels 1..5."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    buf = np.zeros(lib().oq_pred_cap(x.size), dtype=np.uint8)
    n = lib().oq_encode_pred(_dp(x), x.size, level, _u8(buf))
    if n == 0:
        raise ValueError("bad chunk size or level")
    return buf[:n].tobytes()


def pred_symbols(x, level: int):
    """Solution B's symbols in coding order (re parts, then im parts) and
    the number of escapes."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    sym = np.zeros(x.size, dtype=np.uint16)
    nesc = lib().oq_pred_symbols(_dp(x), x.size, level, sym.ctypes.data)
    if nesc < 0:
        raise ValueError("bad level")
    return sym, nesc


def pred_huff_lengths(counts) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint32))
    out = np.zeros(c.size, dtype=np.uint8)
    lib().oq_pred_huff_lengths(c.ctypes.data, c.size, _u8(out))
    return out


def pred_width(level: int) -> int:
    return lib().oq_pred_width(level)


def huff_lengths(counts) -> np.ndarray:
    """Code lengths of the entropy stage's length-limited Huffman code."""
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint32))
    out = np.zeros(c.size, dtype=np.uint8)
    if lib().oq_huff_lengths(c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), c.size, _u8(out)) != 0:
        raise ValueError("need 1..16 symbols, at least two present")
    return out


def canon_codes(lengths) -> np.ndarray:
    ln = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint8))
    out = np.zeros(ln.size, dtype=np.uint32)
    if lib().oq_canon_codes(_u8(ln), ln.size, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))) != 0:
        raise ValueError("bad lengths")
    return out


def decode_chunk(data: bytes, C: int) -> np.ndarray:
    buf = np.frombuffer(bytes(data), dtype=np.uint8).copy()
    out = np.zeros(C, dtype=np.float64)
    if lib().oq_decode_chunk(_u8(buf), buf.size, C, _dp(out)) != 0:
        raise ValueError("malformed chunk")
    return out


# --------------------------------------------------------------------------
# gates
# --------------------------------------------------------------------------
def gate_check(g, n: int) -> bool:
    g = _gates(g)
    return lib().oq_gate_check(g.ctypes.data, n) == 0


def apply_dense(psi: np.ndarray, n: int, gates) -> np.ndarray:
    """Uncompressed fp64 reference: psi (complex128, 2^n) after the gate list."""
    gates = _gates(gates)
    st = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    d = st.view(np.float64)
    L = lib()
    for k in range(len(gates)):
        if L.oq_apply_gate_dense(_dp(d), n, gates[k:k + 1].ctypes.data) != 0:
            raise ValueError("malformed gate %d" % k)
    return st


def chunk_role(g, cb: int, c: int) -> int:
    return lib().oq_chunk_role(_gates(g).ctypes.data, cb, c)


def gate_job(g, cb: int, C: int, c0: int, in0: bytes, level0: int,
             c1: int | None = None, in1: bytes | None = None, level1: int = 0, flags: int = 0):
    """One unit of the blockwise loop on exported chunk bytes (flags: codec
    flags ENC_*)."""
    g = _gates(g)
    cap = chunk_cap(C)
    b0 = np.frombuffer(bytes(in0), dtype=np.uint8).copy()
    o0 = np.zeros(cap, dtype=np.uint8)
    n0 = ctypes.c_size_t(0)
    n1 = ctypes.c_size_t(0)
    if in1 is None:
        rc = lib().oq_gate_job_ex(g.ctypes.data, cb, C, flags, c0, _u8(b0), b0.size, level0, _u8(o0),
                                  ctypes.byref(n0), 0, None, 0, 0, None, None)
        if rc != 0:
            raise ValueError("malformed chunk")
        return o0[:n0.value].tobytes()
    b1 = np.frombuffer(bytes(in1), dtype=np.uint8).copy()
    o1 = np.zeros(cap, dtype=np.uint8)
    rc = lib().oq_gate_job_ex(g.ctypes.data, cb, C, flags, c0, _u8(b0), b0.size, level0, _u8(o0),
                              ctypes.byref(n0), c1, _u8(b1), b1.size, level1, _u8(o1), ctypes.byref(n1))
    if rc != 0:
        raise ValueError("malformed chunk")
    return o0[:n0.value].tobytes(), o1[:n1.value].tobytes()


# --------------------------------------------------------------------------
# compressed simulator
# --------------------------------------------------------------------------
class Sim:
    """Blockwise compressed simulator (Sec. 3.1/3.3) with the Sec. 3.7 rule."""

    def __init__(self, n: int, block_log2: int, mode: int = MODE_LOSSLESS,
                 level: int = 0, budget: int = 0, codec: int = 0):
        self.n, self.block_log2 = n, block_log2
        self._h = lib().oq_sim_create(n, block_log2, mode, level, budget)
        self._destroy = lib().oq_sim_destroy   # held: module globals may be gone when __del__ runs at exit
        if not self._h:
            raise ValueError("bad simulator configuration")
        if codec:
            lib().oq_sim_set_codec(self._h, codec)   # ENC_ENTROPY / ENC_RESHUFFLE for later encodes
        self.cb = lib().oq_sim_chunk_log2(self._h)
        self.C = 2 << self.cb
        self.nchunks = 1 << (n - self.cb)

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def apply(self, gates) -> int:
        gates = _gates(gates)
        if len(gates) == 0:
            return 0
        return lib().oq_sim_apply(self._h, gates.ctypes.data, len(gates))

    def state(self) -> np.ndarray:
        out = np.zeros(2 << self.n, dtype=np.float64)
        if lib().oq_sim_read_all(self._h, _dp(out)) != 0:
            raise RuntimeError("decode failed")
        return out.view(np.complex128)

    def chunk(self, c: int) -> bytes:
        cap = chunk_cap(self.C)
        buf = np.zeros(cap, dtype=np.uint8)
        n = lib().oq_sim_chunk(self._h, c, _u8(buf), cap)
        return buf[:n].tobytes()

    def set_chunk(self, c: int, data: bytes):
        b = np.frombuffer(bytes(data), dtype=np.uint8).copy()
        if lib().oq_sim_set_chunk(self._h, c, _u8(b), b.size) != 0:
            raise ValueError("bad chunk")

    def set_block_level(self, b: int, level: int):
        if lib().oq_sim_set_block_level(self._h, b, level) != 0:
            raise ValueError("bad block/level")

    def footprint(self) -> dict:
        u = (ctypes.c_uint64 * 7)()
        f = (ctypes.c_double * 2)()
        lib().oq_sim_footprint(self._h, u, f)
        return {"compressed_bytes": u[0], "nchunks": u[1], "level": u[2], "gates_applied": u[3],
                "lossy_steps": u[4], "min_compressed": u[5], "max_compressed": u[6],
                "fidelity_lower_bound": f[0], "fidelity_lower_bound_weighted": f[1]}
