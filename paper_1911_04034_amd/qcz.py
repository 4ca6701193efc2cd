"""ctypes binding of libqcz.so (C ABI in include/qcz.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library.  PyTorch provides the device pool and the stream.
Raises RuntimeError when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcz.so")

MODE_LOSSLESS, MODE_FIXED, MODE_ADAPTIVE, MODE_PERBLOCK = 0, 1, 2, 3
FLAG_GRAPH = 1
FLAG_TIMING = 2
FLAG_AUTOTUNE = 4
FLAG_RANGES = 8
FLAG_CACHE = 16
FLAG_CACHE_COLLIDE = 32
FLAG_FUSE = 64
FLAG_ENTROPY = 128
FLAG_RESHUFFLE = 256
FLAG_GROUPS = 512
CODEC_ENTROPY = 1
CODEC_RESHUFFLE = 2
CODEC_PREDICT = 4
STATUS = {0: "QCZ_OK", -1: "QCZ_E_INVAL", -2: "QCZ_E_NOMEM", -3: "QCZ_E_DEVICE", -4: "QCZ_E_FORMAT",
          -5: "QCZ_E_STATE"}


class QczError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_uint32), ("block_log2", ctypes.c_uint32), ("mode", ctypes.c_int32),
                ("level", ctypes.c_int32), ("budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("batch", ctypes.c_uint32), ("grid", ctypes.c_uint32), ("chunk_waves", ctypes.c_uint32),
                ("reserved", ctypes.c_uint64 * 3)]


class Footprint(ctypes.Structure):
    _fields_ = [("compressed_bytes", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64),
                ("total_bytes", ctypes.c_uint64), ("raw_bytes", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("arena_used", ctypes.c_uint64), ("nchunks", ctypes.c_uint64), ("gates_applied", ctypes.c_uint64),
                ("lossy_steps", ctypes.c_uint64), ("min_compressed", ctypes.c_uint64),
                ("max_compressed", ctypes.c_uint64), ("compactions", ctypes.c_uint64), ("level", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ratio", ctypes.c_double),
                ("fidelity_lower_bound", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("gate_launches", ctypes.c_uint64), ("permute_launches", ctypes.c_uint64),
                ("chunks_reencoded", ctypes.c_uint64), ("amps_touched", ctypes.c_uint64),
                ("bytes_read", ctypes.c_uint64), ("bytes_written", ctypes.c_uint64),
                ("table_bytes", ctypes.c_uint64), ("timed_launches", ctypes.c_uint64),
                ("gate_kernel_ms", ctypes.c_double), ("chunk_waves", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("tuning", ctypes.c_uint32), ("stops", ctypes.c_uint32),
                ("range_gates", ctypes.c_uint64), ("cache_gates", ctypes.c_uint64),
                ("cache_hits", ctypes.c_uint64), ("cache_on", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("range_launches", ctypes.c_uint64), ("sweep_gates", ctypes.c_uint64),
                ("kind_launches", ctypes.c_uint64 * 3), ("kind_kernel_ms", ctypes.c_double * 3),
                ("kind_bytes", ctypes.c_uint64 * 3)]


EXPORTED = [
    "qcz_pool_bytes_min", "qcz_create", "qcz_apply_gates", "qcz_read_amplitudes", "qcz_decode_chunks_to",
    "qcz_moments", "qcz_sample", "qcz_footprint", "qcz_export_chunk", "qcz_import_chunk", "qcz_set_block_levels",
    "qcz_chunk_sizes", "qcz_num_chunks", "qcz_chunk_doubles", "qcz_last_error", "qcz_destroy", "qcz_chunk_cap",
    "qcz_chunk_cap_codec",
    "qcz_encode_chunks", "qcz_decode_chunks", "qcz_get_stats", "qcz_reset_stats", "qcz_set_launch",
    "qcz_block_stats", "qcz_block_level_sizes", "qcz_label_levels", "qcz_project_levels", "qcz_mlp_forward",
    "qcz_mlp_workspace_bytes", "qcz_mlp_train_step", "qcz_mlp_train_step_noalloc", "qcz_select_levels", "qcz_set_selector", "qcz_copy_state",
    "qcz_mixing_mask", "qcz_overlap", "qcz_resume", "qcz_export_state", "qcz_import_state",
]
MLP_PARAMS = 5638
N_FEATURES = 16

_lib = None


def load():
    """Load libqcz.so (built in-tree by __graft_entry__.build()).

    torch is imported first: torch brings its own HIP runtime, and libqcz.so
    must bind to that same runtime (loaded first, the system one would be a
    second runtime in the process, with which torch's device memory and
    streams cannot be used)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (see above)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libqcz.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u64, u32, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.qcz_pool_bytes_min.restype = sz
    L.qcz_pool_bytes_min.argtypes = [ctypes.POINTER(Config)]
    L.qcz_create.restype = i32
    L.qcz_create.argtypes = [ctypes.POINTER(Config), vp, sz, vp, ctypes.POINTER(vp)]
    L.qcz_apply_gates.restype = i32
    L.qcz_apply_gates.argtypes = [vp, vp, sz, ctypes.POINTER(sz)]
    L.qcz_read_amplitudes.restype = i32
    L.qcz_read_amplitudes.argtypes = [vp, vp, sz, vp]
    L.qcz_decode_chunks_to.restype = i32
    L.qcz_decode_chunks_to.argtypes = [vp, u64, u64, vp]
    L.qcz_moments.restype = i32
    L.qcz_moments.argtypes = [vp, vp]
    L.qcz_sample.restype = i32
    L.qcz_sample.argtypes = [vp, u64, sz, vp]
    L.qcz_footprint.restype = i32
    L.qcz_footprint.argtypes = [vp, ctypes.POINTER(Footprint)]
    L.qcz_resume.argtypes = [vp, ctypes.POINTER(Footprint)]
    L.qcz_export_state.argtypes = [vp, vp, sz, vp, ctypes.POINTER(sz)]
    L.qcz_import_state.argtypes = [vp, vp, sz, vp]
    L.qcz_export_chunk.restype = i32
    L.qcz_export_chunk.argtypes = [vp, u64, vp, sz, ctypes.POINTER(sz)]
    L.qcz_import_chunk.restype = i32
    L.qcz_import_chunk.argtypes = [vp, u64, vp, sz]
    L.qcz_set_block_levels.restype = i32
    L.qcz_set_block_levels.argtypes = [vp, vp]
    L.qcz_chunk_sizes.restype = i32
    L.qcz_chunk_sizes.argtypes = [vp, vp]
    L.qcz_num_chunks.restype = u64
    L.qcz_num_chunks.argtypes = [vp]
    L.qcz_chunk_doubles.restype = u32
    L.qcz_chunk_doubles.argtypes = [vp]
    L.qcz_last_error.restype = ctypes.c_char_p
    L.qcz_last_error.argtypes = [vp]
    L.qcz_destroy.restype = None
    L.qcz_destroy.argtypes = [vp]
    L.qcz_chunk_cap.restype = sz
    L.qcz_chunk_cap.argtypes = [u32]
    L.qcz_chunk_cap_codec.restype = sz
    L.qcz_chunk_cap_codec.argtypes = [u32, u32]
    L.qcz_encode_chunks.restype = i32
    L.qcz_encode_chunks.argtypes = [vp, u32, u64, i32, u32, vp, sz, vp, vp]
    L.qcz_decode_chunks.restype = i32
    L.qcz_decode_chunks.argtypes = [vp, sz, vp, u32, u64, vp, vp]
    L.qcz_get_stats.restype = i32
    L.qcz_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.qcz_reset_stats.restype = i32
    L.qcz_reset_stats.argtypes = [vp]
    L.qcz_set_launch.restype = i32
    L.qcz_set_launch.argtypes = [vp, u32, u32]
    dbl, flt = ctypes.c_double, ctypes.c_float
    L.qcz_block_stats.restype = i32
    L.qcz_block_stats.argtypes = [vp, dbl, u64, vp, vp]
    L.qcz_block_level_sizes.restype = i32
    L.qcz_block_level_sizes.argtypes = [vp, vp]
    L.qcz_label_levels.restype = i32
    L.qcz_label_levels.argtypes = [vp, vp, u64, dbl, u64, vp]
    L.qcz_project_levels.restype = i32
    L.qcz_project_levels.argtypes = [vp, u64, dbl, u64, vp]
    L.qcz_mlp_forward.restype = i32
    L.qcz_mlp_forward.argtypes = [vp, vp, u64, vp, vp, vp]
    L.qcz_mlp_workspace_bytes.restype = sz
    L.qcz_mlp_workspace_bytes.argtypes = [u64]
    L.qcz_mlp_train_step.restype = i32
    L.qcz_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, u64, flt, u32, vp, vp, vp, sz, vp]
    L.qcz_mlp_train_step_noalloc.restype = i32
    L.qcz_mlp_train_step_noalloc.argtypes = [vp, vp, vp, vp, vp, u64, flt, u32, vp, vp, vp]
    L.qcz_select_levels.restype = i32
    L.qcz_select_levels.argtypes = [vp, vp, dbl, u64, vp]
    L.qcz_set_selector.restype = i32
    L.qcz_set_selector.argtypes = [vp, vp, dbl, u32]
    L.qcz_copy_state.restype = i32
    L.qcz_copy_state.argtypes = [vp, vp]
    L.qcz_mixing_mask.restype = u64
    L.qcz_mixing_mask.argtypes = [vp, vp, sz]
    L.qcz_overlap.restype = i32
    L.qcz_overlap.argtypes = [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    _lib = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible")
    return torch


def chunk_cap(C: int) -> int:
    return load().qcz_chunk_cap(C)


def _gates(g):
    g = np.ascontiguousarray(g)
    if g.dtype.itemsize != 88:
        raise ValueError("gate records must be 88-byte structs (circuits.GATE_DTYPE)")
    return g


class State:
    """A compressed 2^n-amplitude state on the current HIP device."""

    def __init__(self, n: int, block_log2: int, mode: int = MODE_LOSSLESS, level: int = 0, budget: int = 0,
                 pool_bytes: int | None = None, flags: int = 0, batch: int = 0, grid: int = 0, stream=None,
                 chunk_waves: int = 0):
        torch = _torch()
        L = load()
        self._lib = L
        self.n, self.block_log2 = n, block_log2
        cfg = Config(n, block_log2, mode, level, budget, flags, batch, grid, chunk_waves)
        self.cfg = cfg
        pmin = L.qcz_pool_bytes_min(ctypes.byref(cfg))
        if pmin == 0:
            raise QczError(-1, "bad configuration")
        if pool_bytes is None:
            raw = 16 << n
            free, _total = torch.cuda.mem_get_info()
            pool_bytes = max(pmin, min(2 * raw + (256 << 20), int(0.85 * free)))
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        rc = L.qcz_create(ctypes.byref(cfg), self.pool.data_ptr(), int(pool_bytes), self.stream.cuda_stream,
                          ctypes.byref(h))
        if rc != 0:
            raise QczError(rc, "qcz_create failed")
        self._h = h
        self.nchunks = L.qcz_num_chunks(h)
        self.C = L.qcz_chunk_doubles(h)
        self.cb = (self.C // 2).bit_length() - 1

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.qcz_destroy(self._h)
            self._h = None
            self.pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            msg = self._lib.qcz_last_error(self._h)
            raise QczError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    # -- the hot path -----------------------------------------------------
    def apply(self, gates) -> int:
        """Apply gate records; returns the number applied (raises on error)."""
        g = _gates(gates)
        applied = ctypes.c_size_t(0)
        rc = self._lib.qcz_apply_gates(self._h, g.ctypes.data, len(g), ctypes.byref(applied))
        self.last_applied = applied.value
        self._check(rc, "qcz_apply_gates (applied %d)" % applied.value)
        return applied.value

    def try_apply(self, gates):
        """Like apply, but returns (status, applied) instead of raising."""
        g = _gates(gates)
        applied = ctypes.c_size_t(0)
        rc = self._lib.qcz_apply_gates(self._h, g.ctypes.data, len(g), ctypes.byref(applied))
        return rc, applied.value

    # -- readout ----------------------------------------------------------
    def read(self, idx) -> np.ndarray:
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64).reshape(-1))
        out = np.zeros(2 * idx.size, dtype=np.float64)
        self._check(self._lib.qcz_read_amplitudes(self._h, idx.ctypes.data, idx.size, out.ctypes.data),
                    "qcz_read_amplitudes")
        return out.view(np.complex128)

    def decode_to(self, first_chunk: int, n_chunks: int, dev_tensor):
        self._check(self._lib.qcz_decode_chunks_to(self._h, first_chunk, n_chunks, dev_tensor.data_ptr()),
                    "qcz_decode_chunks_to")

    def state(self) -> np.ndarray:
        """Whole decoded state as complex128 (host)."""
        torch = _torch()
        out = torch.empty(self.nchunks * self.C, dtype=torch.float64, device="cuda")
        self.decode_to(0, self.nchunks, out)
        return out.cpu().numpy().view(np.complex128)

    def moments(self):
        out = np.zeros(3, dtype=np.float64)
        self._check(self._lib.qcz_moments(self._h, out.ctypes.data), "qcz_moments")
        return complex(out[0], out[1]), float(out[2])

    def footprint(self) -> dict:
        f = Footprint()
        self._check(self._lib.qcz_footprint(self._h, ctypes.byref(f)), "qcz_footprint")
        return {k: getattr(f, k) for k, _ in Footprint._fields_ if k != "reserved"}

    def stats(self) -> dict:
        st = Stats()
        self._check(self._lib.qcz_get_stats(self._h, ctypes.byref(st)), "qcz_get_stats")
        out = {}
        for k, _ in Stats._fields_:
            v = getattr(st, k)
            out[k] = list(v) if k.startswith("kind_") else v
        return out

    def reset_stats(self):
        self._check(self._lib.qcz_reset_stats(self._h), "qcz_reset_stats")

    def set_launch(self, chunk_waves: int = 0, grid: int = 0):
        self._check(self._lib.qcz_set_launch(self._h, chunk_waves, grid), "qcz_set_launch")

    def export_chunk(self, c: int) -> bytes:
        cap = chunk_cap(self.C)
        buf = np.zeros(cap, dtype=np.uint8)
        ln = ctypes.c_size_t(0)
        self._check(self._lib.qcz_export_chunk(self._h, c, buf.ctypes.data, cap, ctypes.byref(ln)),
                    "qcz_export_chunk")
        return buf[:ln.value].tobytes()

    def import_chunk(self, c: int, data: bytes):
        b = np.frombuffer(bytes(data), dtype=np.uint8).copy()
        self._check(self._lib.qcz_import_chunk(self._h, c, b.ctypes.data, b.size), "qcz_import_chunk")

    # -- checkpoint / resume (Sec. 3.5) --------------------------------------
    def export_state(self):
        """(image, sizes): every chunk's stream in chunk order, each padded to
        16 bytes, as one host array (the state is compacted first)."""
        sizes = np.zeros(self.nchunks, dtype=np.uint32)
        total = ctypes.c_size_t(0)
        self._check(self._lib.qcz_export_state(self._h, None, 0, sizes.ctypes.data, ctypes.byref(total)),
                    "qcz_export_state")
        image = np.zeros(max(1, total.value), dtype=np.uint8)
        self._check(self._lib.qcz_export_state(self._h, image.ctypes.data, image.size, sizes.ctypes.data,
                                               ctypes.byref(total)), "qcz_export_state")
        return image[:total.value], sizes

    def import_state(self, image, sizes):
        image = np.ascontiguousarray(image, dtype=np.uint8)
        sizes = np.ascontiguousarray(sizes, dtype=np.uint32)
        if sizes.size != self.nchunks:
            raise QczError(-1, "one size per chunk expected")
        self._check(self._lib.qcz_import_state(self._h, image.ctypes.data, image.size, sizes.ctypes.data),
                    "qcz_import_state")

    def save(self, path: str):
        """Write the compressed chunks and the ledger to `path` (.npz: plain
        arrays, loadable without pickle)."""
        image, sizes = self.export_state()
        fp = Footprint()
        self._check(self._lib.qcz_footprint(self._h, ctypes.byref(fp)), "qcz_footprint")
        cfg = np.array([self.cfg.n_qubits, self.cfg.block_log2, self.cfg.mode, self.cfg.level, self.cfg.budget_bytes,
                        self.cfg.flags, self.cfg.batch, self.cfg.grid, self.cfg.chunk_waves], dtype=np.int64)
        np.savez(path, config=cfg, sizes=sizes, streams=image, footprint=np.frombuffer(bytes(fp), dtype=np.uint8))

    @classmethod
    def load(cls, path: str, pool_bytes: int | None = None, stream=None) -> "State":
        """A new state holding the chunks and ledger saved by `save`."""
        with np.load(path, allow_pickle=False) as z:
            cfg, sizes, streams, fpb = z["config"], z["sizes"], z["streams"], z["footprint"]
        n, bl, mode, level, budget, flags, batch, grid, waves = (int(v) for v in cfg)
        st = cls(n, bl, mode=mode, level=level, budget=budget, pool_bytes=pool_bytes, flags=flags, batch=batch,
                 grid=grid, stream=stream, chunk_waves=waves)
        if sizes.size != st.nchunks or fpb.size != ctypes.sizeof(Footprint):
            raise QczError(-1, "checkpoint does not match the configuration")
        st.import_state(streams, sizes)
        fp = Footprint.from_buffer_copy(fpb.tobytes())
        st._check(st._lib.qcz_resume(st._h, ctypes.byref(fp)), "qcz_resume")
        return st

    def chunk_sizes(self) -> np.ndarray:
        out = np.zeros(self.nchunks, dtype=np.uint32)
        self._check(self._lib.qcz_chunk_sizes(self._h, out.ctypes.data), "qcz_chunk_sizes")
        return out

    def set_block_levels(self, levels):
        lv = np.ascontiguousarray(np.asarray(levels, dtype=np.uint8))
        self._check(self._lib.qcz_set_block_levels(self._h, lv.ctypes.data), "qcz_set_block_levels")

    # -- per-block level selection -------------------------------------------
    def block_stats(self, beta: float, mask: int = 0):
        """(features float32 [nblocks, 16], squared norms float64 [nblocks]) on the device."""
        torch = _torch()
        nb = 1 << (self.n - self.block_log2)
        X = torch.empty((nb, N_FEATURES), dtype=torch.float32, device="cuda")
        n2 = torch.empty(nb, dtype=torch.float64, device="cuda")
        self._check(self._lib.qcz_block_stats(self._h, float(beta), int(mask), X.data_ptr(), n2.data_ptr()),
                    "qcz_block_stats")
        return X, n2

    def block_level_sizes(self):
        """Padded bytes of every block at each level: int64 [nblocks, 6] on the device."""
        torch = _torch()
        nb = 1 << (self.n - self.block_log2)
        S = torch.empty((nb, 6), dtype=torch.int64, device="cuda")
        self._check(self._lib.qcz_block_level_sizes(self._h, S.data_ptr()), "qcz_block_level_sizes")
        return S

    def select_levels(self, params, beta: float, mask: int = 0) -> np.ndarray:
        nb = 1 << (self.n - self.block_log2)
        out = np.zeros(nb, dtype=np.uint8)
        self._check(self._lib.qcz_select_levels(self._h, params.data_ptr(), float(beta), int(mask), out.ctypes.data),
                    "qcz_select_levels")
        return out

    def set_selector(self, params, beta: float = 0.0, period: int = 1):
        """Attach (params: cuda float32 [5638], kept alive here) or detach (None)."""
        self._sel_params = params
        ptr = params.data_ptr() if params is not None else None
        self._check(self._lib.qcz_set_selector(self._h, ptr, float(beta), int(period)), "qcz_set_selector")

    def copy_from(self, src: "State"):
        """Make this state equal to src (same n, block size and mode)."""
        self._check(self._lib.qcz_copy_state(self._h, src._h), "qcz_copy_state")

    def mixing_mask(self, gates) -> int:
        g = _gates(gates)
        return int(self._lib.qcz_mixing_mask(self._h, g.ctypes.data, len(g)))

    def overlap(self, other: "State") -> complex:
        """<self|other> over the decoded states."""
        re, im = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(self._lib.qcz_overlap(self._h, other._h, ctypes.byref(re), ctypes.byref(im)), "qcz_overlap")
        return complex(re.value, im.value)

    def sample(self, seed: int, shots: int) -> np.ndarray:
        out = np.zeros(shots, dtype=np.uint64)
        self._check(self._lib.qcz_sample(self._h, seed, shots, out.ctypes.data), "qcz_sample")
        return out


# -- codec entry points -----------------------------------------------------
def encode_chunks(x, level: int, stream=None, codec_flags: int = 0):
    """x: cuda float64 tensor [n, C].  Returns (slots uint8 [n, slot], sizes).
    codec_flags: CODEC_ENTROPY lets chunks take the entropy-coded body,
    CODEC_RESHUFFLE stores Solution D's order, CODEC_PREDICT (alone) encodes
    with Solution B."""
    torch = _torch()
    L = load()
    n, C = x.shape
    cap = L.qcz_chunk_cap_codec(C, codec_flags)
    if cap == 0:
        raise QczError(-1, "qcz_chunk_cap_codec")
    slot = (cap + 3) & ~3
    slots = torch.zeros((n, slot), dtype=torch.uint8, device=x.device)
    sizes = torch.zeros(n, dtype=torch.int32, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = L.qcz_encode_chunks(x.contiguous().data_ptr(), C, n, level, codec_flags, slots.data_ptr(), slot,
                             sizes.data_ptr(), st.cuda_stream)
    if rc != 0:
        raise QczError(rc, "qcz_encode_chunks")
    st.synchronize()
    return slots, sizes


def decode_chunks(slots, sizes, C: int, stream=None):
    torch = _torch()
    L = load()
    n, slot = slots.shape
    out = torch.empty((n, C), dtype=torch.float64, device=slots.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = L.qcz_decode_chunks(slots.data_ptr(), slot, sizes.data_ptr(), C, n, out.data_ptr(), st.cuda_stream)
    if rc != 0:
        raise QczError(rc, "qcz_decode_chunks")
    st.synchronize()
    return out


# -- selector entry points ----------------------------------------------------
def label_levels(sizes, w, beta: float, mask: int = 0) -> np.ndarray:
    """Host call: Lagrangian level labels (sizes [nblocks, 6] u64, w [nblocks])."""
    S = np.ascontiguousarray(np.asarray(sizes, dtype=np.uint64))
    W = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    out = np.zeros(W.size, dtype=np.uint8)
    rc = load().qcz_label_levels(S.ctypes.data, W.ctypes.data, W.size, float(beta), int(mask), out.ctypes.data)
    if rc != 0:
        raise QczError(rc, "qcz_label_levels")
    return out


def project_levels(levels, w, beta: float, mask: int = 0) -> np.ndarray:
    """Host call: budget projection of per-block levels."""
    L = np.ascontiguousarray(np.asarray(levels, dtype=np.uint8)).copy()
    W = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    rc = load().qcz_project_levels(W.ctypes.data, W.size, float(beta), int(mask), L.ctypes.data)
    if rc != 0:
        raise QczError(rc, "qcz_project_levels")
    return L


def mlp_forward(params, X, stream=None):
    """(probabilities float32 [N, 6], levels uint8 [N]) for features X (cuda float32 [N, 16])."""
    torch = _torch()
    N = X.shape[0]
    probs = torch.empty((N, 6), dtype=torch.float32, device=X.device)
    lev = torch.empty(N, dtype=torch.uint8, device=X.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = load().qcz_mlp_forward(params.data_ptr(), X.contiguous().data_ptr(), N, probs.data_ptr(), lev.data_ptr(),
                                st.cuda_stream)
    if rc != 0:
        raise QczError(rc, "qcz_mlp_forward")
    st.synchronize()
    return probs, lev


class MLPTrainer:
    """Device-resident parameters, Adam moments and workspace of the selector."""

    def __init__(self, params, n_samples: int, stream=None):
        torch = _torch()
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grad = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.n = int(n_samples)
        self.work = torch.empty(load().qcz_mlp_workspace_bytes(self.n), dtype=torch.uint8, device=params.device)
        self.t = 0
        self.stream = stream if stream is not None else torch.cuda.current_stream()

    def step(self, X, labels, lr: float, update: bool = True, sync: bool = True):
        """One full-batch step (update=False: loss and gradient only)."""
        assert X.shape[0] == self.n and labels.shape[0] == self.n
        if update:
            self.t += 1
        rc = load().qcz_mlp_train_step(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), X.data_ptr(),
                                       labels.data_ptr(), self.n, float(lr), self.t if update else 0,
                                       self.grad.data_ptr(), self.loss.data_ptr(), self.work.data_ptr(),
                                       self.work.numel(), self.stream.cuda_stream)
        if rc != 0:
            raise QczError(rc, "qcz_mlp_train_step")
        if sync:
            self.stream.synchronize()
            return float(self.loss.item())
        return None
