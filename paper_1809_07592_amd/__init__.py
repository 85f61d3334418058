"""MI355X-native Toeplitz-hash privacy amplification.

Thin ctypes binding over ``libpa.so`` (C ABI in ``include/pa.h``): it only
marshals torch CUDA tensors (device memory) and HIP streams into the C
calls; every step of the hash runs in the library's gfx950 kernels.  The
library is built in-tree by ``python -m paper_1809_07592_amd.build``; if it is
missing, every call raises ``RuntimeError`` (there is no fallback).

Bit tensors are int64 (or uint64) CUDA tensors holding little-endian packed
bits: bit k in word k >> 6 at position k & 63.
"""
from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpa.so")

PA_OK = 0
PA_ERR_INVALID_ARG = 1
PA_ERR_UNSUPPORTED_SIZE = 2
PA_ERR_OUT_OF_MEMORY = 3
PA_ERR_DEVICE = 4
PA_ERR_BUSY = 5
PA_ERR_CANCELLED = 6
MAX_TRANSFORM_LEN = 28311552

_lib = None
_lock = threading.Lock()


class PAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (status_string(status) if _lib else status, message))
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [("transform_len", ctypes.c_uint64), ("rows", ctypes.c_uint32), ("cols", ctypes.c_uint32),
                ("tile_width", ctypes.c_uint32), ("col_tiles", ctypes.c_uint32), ("col_threads", ctypes.c_uint32),
                ("row_threads", ctypes.c_uint32), ("col_lds_bytes", ctypes.c_uint32),
                ("row_lds_bytes", ctypes.c_uint32), ("col_rounds", ctypes.c_uint32), ("row_rounds", ctypes.c_uint32),
                ("col_round_size", ctypes.c_uint32 * 6), ("row_round_size", ctypes.c_uint32 * 6),
                ("row_shape", ctypes.c_uint32), ("col_shape", ctypes.c_uint32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["col_round_size"] = list(self.col_round_size)[: self.col_rounds]
        d["row_round_size"] = list(self.row_round_size)[: self.row_rounds]
        return d


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("alg_ops", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("max_queue", ctypes.c_uint32), ("streams", ctypes.c_uint32), ("executor", ctypes.c_uint32),
                ("sim_bits_per_us", ctypes.c_double), ("sim_fail_every", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "submitted", "completed", "rejected", "batches", "bytes_in_flight", "peak_bytes_in_flight",
        "budget_bytes", "inflight", "peak_inflight", "pending", "input_bits_completed", "spectrum_bytes",
        "spectra_resident", "spectra_built", "spectra_evicted", "cancelled", "failed")]


class TuneResult(ctypes.Structure):
    _fields_ = [("log2_rows", ctypes.c_uint32), ("tile_width", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
                ("count", ctypes.c_uint32), ("best_us", ctypes.c_double), ("default_us", ctypes.c_double),
                ("row_first", ctypes.c_uint32), ("row_threads", ctypes.c_uint32)]


class PhaseProbeResult(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_uint32), ("threads", ctypes.c_uint32), ("phase_bytes", ctypes.c_double),
                ("empty_launch_us", ctypes.c_double), ("empty_cooperative_us", ctypes.c_double),
                ("three_launches_us", ctypes.c_double), ("cooperative_grid_sync_us", ctypes.c_double),
                ("tiles", ctypes.c_uint32), ("tiles_no_release_us", ctypes.c_double),
                ("tiles_release_us", ctypes.c_double)]


class TuneGeometry(ctypes.Structure):
    _fields_ = [("log2_rows", ctypes.c_uint32), ("tile_width", ctypes.c_uint32), ("row_first", ctypes.c_uint32),
                ("row_threads", ctypes.c_uint32)]


class _Block(ctypes.Structure):
    _fields_ = [("key_bits", ctypes.c_void_p), ("n", ctypes.c_uint64), ("seed_bits", ctypes.c_void_p),
                ("m", ctypes.c_uint64), ("out_bits", ctypes.c_void_p)]


def lib():
    """The loaded libpa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError("libpa.so is not built (run: python -m paper_1809_07592_amd.build); "
                                       "there is no CPU fallback")
                # torch ships its own HIP runtime under the soname libpa
                # needs; the first one loaded serves the whole process, and
                # torch fails on any other, so it is loaded first
                try:
                    import torch  # noqa: F401
                except ImportError:
                    pass
                L = ctypes.CDLL(LIB_PATH)
                vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
                st = ctypes.c_int
                L.pa_toeplitz_hash.argtypes = [vp, u64, vp, u64, vp, vp]
                L.pa_toeplitz_hash.restype = st
                L.pa_toeplitz_hash_noalloc.argtypes = [vp, u64, vp, u64, vp, vp]
                L.pa_toeplitz_hash_noalloc.restype = st
                L.pa_toeplitz_hash_batched.argtypes = [ctypes.POINTER(_Block), u32, vp]
                L.pa_toeplitz_hash_batched.restype = st
                L.pa_plan_create.argtypes = [vp, u64, u64, vp, ctypes.POINTER(vp)]
                L.pa_plan_create.restype = st
                L.pa_plan_hash.argtypes = [vp, vp, u64, u64, vp, vp]
                L.pa_plan_hash.restype = st
                L.pa_plan_transform_len.argtypes = [vp]
                L.pa_plan_transform_len.restype = u64
                L.pa_plan_destroy.argtypes = [vp]
                L.pa_plan_destroy.restype = st
                L.pa_transform_len.argtypes = [u64, u64]
                L.pa_transform_len.restype = u64
                L.pa_plan_describe.argtypes = [u64, u32, u32, ctypes.POINTER(PlanInfo)]
                L.pa_plan_describe.restype = st
                L.pa_modified_toeplitz_hash.argtypes = [vp, u64, vp, u64, vp, vp]
                L.pa_modified_toeplitz_hash.restype = st
                L.pa_modified_toeplitz_hash_batched.argtypes = [ctypes.POINTER(_Block), u32, vp]
                L.pa_modified_toeplitz_hash_batched.restype = st
                L.pa_graph_create.argtypes = [ctypes.POINTER(_Block), u32, ctypes.c_int, ctypes.POINTER(vp)]
                L.pa_graph_create.restype = st
                L.pa_graph_launch.argtypes = [vp, vp]
                L.pa_graph_launch.restype = st
                L.pa_graph_update.argtypes = [vp, ctypes.POINTER(_Block), u32, vp]
                L.pa_graph_update.restype = st
                L.pa_graph_block_count.argtypes = [vp]
                L.pa_graph_block_count.restype = u32
                L.pa_graph_destroy.argtypes = [vp]
                L.pa_graph_destroy.restype = st
                L.pa_fft_pair_transform_len.argtypes = [u64, u64]
                L.pa_fft_pair_transform_len.restype = u64
                L.pa_toeplitz_hash_pair_fft.argtypes = [vp, vp, u64, vp, u64, vp, vp, ctypes.c_double, vp,
                                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
                L.pa_toeplitz_hash_pair_fft.restype = st
                L.pa_alu_probe.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
                L.pa_alu_probe.restype = st
                L.pa_launch_probe.argtypes = [vp, u32, u32, u32, ctypes.POINTER(ctypes.c_double)]
                L.pa_launch_probe.restype = st
                L.pa_phase_probe.argtypes = [vp, ctypes.POINTER(PhaseProbeResult)]
                L.pa_phase_probe.restype = st
                L.pa_final_key_length.argtypes = [u64, u64, u64]
                L.pa_final_key_length.restype = u64
                L.pa_cyclic_convolution.argtypes = [vp, u64, vp, u64, u64, vp, vp]
                L.pa_cyclic_convolution.restype = st
                L.pa_plan_spectrum.argtypes = [vp, vp, vp]
                L.pa_plan_spectrum.restype = st
                L.pa_tune_set_geometry.argtypes = [u64, u32, ctypes.POINTER(TuneGeometry)]
                L.pa_tune_set_geometry.restype = st
                L.pa_tune_get_geometry.argtypes = [u64, u32, ctypes.POINTER(TuneGeometry)]
                L.pa_tune_get_geometry.restype = st
                L.pa_tune_set.argtypes = [u64, u32, u32, u32]
                L.pa_tune_set.restype = st
                L.pa_tune_get.argtypes = [u64, u32, ctypes.POINTER(u32), ctypes.POINTER(u32)]
                L.pa_tune_get.restype = st
                L.pa_autotune.argtypes = [u64, u32, u32, vp, ctypes.POINTER(TuneResult)]
                L.pa_autotune.restype = st
                L.pa_tune_save.argtypes = [ctypes.c_char_p]
                L.pa_tune_save.restype = st
                L.pa_tune_load.argtypes = [ctypes.c_char_p]
                L.pa_tune_load.restype = st
                L.pa_profile_enable.argtypes = [ctypes.c_int]
                L.pa_profile_enable.restype = st
                L.pa_profile_collect.argtypes = [ctypes.POINTER(KernelStat), u32, ctypes.POINTER(u32)]
                L.pa_profile_collect.restype = st
                vpp = ctypes.POINTER(vp)
                L.pa_server_create.argtypes = [ctypes.POINTER(ServerConfig), vpp]
                L.pa_server_create.restype = st
                L.pa_server_register_seed.argtypes = [vp, vp, u64, ctypes.POINTER(u32)]
                L.pa_server_register_seed.restype = st
                L.pa_server_submit.argtypes = [vp, u32, vp, u64, u64, vp, ctypes.POINTER(u64)]
                L.pa_server_submit.restype = st
                L.pa_server_poll.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int)]
                L.pa_server_poll.restype = st
                L.pa_server_cancel.argtypes = [vp, u64]
                L.pa_server_cancel.restype = st
                L.pa_server_wait.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double)]
                L.pa_server_wait.restype = st
                L.pa_server_drain.argtypes = [vp]
                L.pa_server_drain.restype = st
                L.pa_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
                L.pa_server_stats_get.restype = st
                L.pa_server_latency.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double)]
                L.pa_server_latency.restype = st
                L.pa_server_destroy.argtypes = [vp]
                L.pa_server_destroy.restype = st
                L.pa_workspace_bytes.argtypes = [u64, u64]
                L.pa_workspace_bytes.restype = ctypes.c_size_t
                L.pa_status_string.argtypes = [st]
                L.pa_status_string.restype = ctypes.c_char_p
                L.pa_last_error.argtypes = []
                L.pa_last_error.restype = ctypes.c_char_p
                L.pa_version.argtypes = []
                L.pa_version.restype = ctypes.c_char_p
                _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().pa_status_string(int(status)).decode()


def last_error() -> str:
    return lib().pa_last_error().decode()


def version() -> str:
    return lib().pa_version().decode()


def _check(status: int):
    if status != PA_OK:
        raise PAError(status, last_error())


def words(bits: int) -> int:
    return (int(bits) + 63) // 64


def transform_len(n: int, m: int) -> int:
    return int(lib().pa_transform_len(int(n), int(m)))


def plan_info(transform_len: int, log2_rows: int = 0, tile_width: int = 0) -> dict:
    """Launch geometry of a transform length (no device work)."""
    info = PlanInfo()
    _check(lib().pa_plan_describe(int(transform_len), int(log2_rows), int(tile_width), ctypes.byref(info)))
    return info.as_dict()


def tune_set(transform_len: int, batch_class: int, log2_rows: int, tile_width: int, row_first: int = 0,
             row_threads: int = 0):
    """Use this geometry for the length in batch class 0 (one block per
    launch) or 1 (several): the (R, W) split, the row transform's first
    round split and a fixed row workgroup size; all zero restores the
    default."""
    g = TuneGeometry(int(log2_rows), int(tile_width), int(row_first), int(row_threads))
    _check(lib().pa_tune_set_geometry(int(transform_len), int(batch_class), ctypes.byref(g)))


def tune_get(transform_len: int, batch_class: int) -> tuple:
    """(log2_rows, tile_width) in effect for the length and class."""
    a, w = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().pa_tune_get(int(transform_len), int(batch_class), ctypes.byref(a), ctypes.byref(w)))
    return int(a.value), int(w.value)


def tune_get_geometry(transform_len: int, batch_class: int) -> dict:
    """The full geometry in effect for the length and class."""
    g = TuneGeometry()
    _check(lib().pa_tune_get_geometry(int(transform_len), int(batch_class), ctypes.byref(g)))
    return {f: int(getattr(g, f)) for f, _ in g._fields_}


def autotune(transform_len: int, count: int = 1, reps: int = 5, stream=None) -> dict:
    """Time the valid geometries of the length on `count` synthetic blocks
    (every (R, W) split, then the row round splits and row workgroup sizes
    at the best) and install the fastest for that batch class."""
    r = TuneResult()
    _check(lib().pa_autotune(int(transform_len), int(count), int(reps), _stream_handle(stream), ctypes.byref(r)))
    return {"log2_rows": int(r.log2_rows), "tile_width": int(r.tile_width), "row_first": int(r.row_first),
            "row_threads": int(r.row_threads), "candidates": int(r.candidates), "count": int(r.count),
            "best_us": r.best_us, "default_us": r.default_us}


def tune_save(path: str):
    _check(lib().pa_tune_save(os.fsencode(path)))


def tune_load(path: str):
    _check(lib().pa_tune_load(os.fsencode(path)))


def profile_enable(on: bool = True):
    """Bracket every library kernel launch with HIP events on its stream."""
    _check(lib().pa_profile_enable(1 if on else 0))


def profile_collect() -> dict:
    """{kernel: {launches, total_ms, avg_ms, alg_bytes, alg_ops}}; clears the record."""
    cap = 32
    arr = (KernelStat * cap)()
    n = ctypes.c_uint32()
    _check(lib().pa_profile_collect(arr, cap, ctypes.byref(n)))
    out = {}
    for i in range(min(n.value, cap)):
        k = arr[i]
        out[k.name.decode()] = {"launches": int(k.launches), "total_ms": k.total_ms,
                                "avg_ms": k.total_ms / max(int(k.launches), 1),
                                "alg_bytes": k.alg_bytes, "alg_ops": k.alg_ops}
    return out


def supported_lengths():
    out = []
    for k in range(7, 21):
        for j in range(4):
            L = 2**k * 3**j
            if 4096 <= L <= MAX_TRANSFORM_LEN:
                out.append(L)
    return sorted(out)


def workspace_bytes(n: int, m: int) -> int:
    return int(lib().pa_workspace_bytes(int(n), int(m)))


def _stream_handle(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


_BIT_DTYPES = None


def _bit_dtypes():
    global _BIT_DTYPES
    if _BIT_DTYPES is None:
        import torch
        _BIT_DTYPES = frozenset({torch.int64, getattr(torch, "uint64", torch.int64)})
    return _BIT_DTYPES


def _ptr(t, nwords: int, what: str):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device (CUDA/HIP) tensor" % what)
    if t.dtype not in _bit_dtypes():
        raise ValueError("%s must be int64/uint64 packed bits" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() < nwords:
        raise ValueError("%s has %d words, needs %d" % (what, t.numel(), nwords))
    return t.data_ptr()


def _blocks(blocks, seed_words):
    """ctypes array of pa_block from (key, n, seed, m, out) tuples."""
    arr = (_Block * max(len(blocks), 1))()
    for i, (key, n, seed, m, out) in enumerate(blocks):
        n, m = int(n), int(m)
        b = arr[i]
        b.key_bits = _ptr(key, (n + 63) >> 6, "key")
        b.n = n
        b.seed_bits = _ptr(seed, seed_words(n, m), "seed")
        b.m = m
        b.out_bits = _ptr(out, (m + 63) >> 6, "out")
    return arr


def toeplitz_hash(key, n: int, seed, m: int, out=None, stream=None):
    """y = T x mod 2 (m x n Toeplitz matrix of the n+m-1 seed bits); returns out."""
    import torch
    if out is None:
        out = torch.empty(max(words(m), 1), dtype=torch.int64, device=key.device)
    _check(lib().pa_toeplitz_hash(_ptr(key, words(n), "key"), int(n), _ptr(seed, words(n + m - 1), "seed"),
                                  int(m), _ptr(out, words(m), "out"), _stream_handle(stream)))
    return out


def toeplitz_hash_noalloc(key, n: int, seed, m: int, out, stream=None):
    """pa_toeplitz_hash_noalloc: y = T x mod 2 with the library's static
    device scratch (no allocation; the caller provides out).  The transform
    tables of the block's length must exist on the device (any earlier
    toeplitz_hash call of that transform length builds them)."""
    _check(lib().pa_toeplitz_hash_noalloc(_ptr(key, words(n), "key"), int(n), _ptr(seed, words(n + m - 1), "seed"),
                                          int(m), _ptr(out, words(m), "out"), _stream_handle(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 113246208


def cyclic_convolution(a, na: int, b, nb: int, transform_len: int, out=None, stream=None):
    """pa_cyclic_convolution: the exact length-L cyclic convolution of two
    bit strings (int32 tensor of L values), computed by the hash's passes."""
    import torch
    L = int(transform_len)
    if out is None:
        out = torch.empty(L, dtype=torch.int32, device=a.device)
    if not out.is_cuda or out.dtype != torch.int32 or not out.is_contiguous() or out.numel() < L:
        raise ValueError("out must be a contiguous int32 device tensor of transform_len values")
    _check(lib().pa_cyclic_convolution(_ptr(a, words(na), "a"), int(na), _ptr(b, words(nb), "b"), int(nb), L,
                                       out.data_ptr(), _stream_handle(stream)))
    return out


def toeplitz_hash_batched(blocks, stream=None):
    """blocks: sequence of (key, n, seed, m, out) tuples; returns the outs."""
    arr = _blocks(blocks, lambda n, m: (n + m + 62) >> 6)
    _check(lib().pa_toeplitz_hash_batched(arr, len(blocks), _stream_handle(stream)))
    return [b[4] for b in blocks]


def modified_toeplitz_hash(key, n: int, v, m: int, out=None, stream=None):
    """y = x[0:m] ^ V x[m:n] (V: m x (n-m) Toeplitz of the n-1 bits v); returns out."""
    import torch
    if out is None:
        out = torch.empty(max(words(m), 1), dtype=torch.int64, device=key.device)
    _check(lib().pa_modified_toeplitz_hash(_ptr(key, words(n), "key"), int(n), _ptr(v, words(n - 1), "v"),
                                           int(m), _ptr(out, words(m), "out"), _stream_handle(stream)))
    return out


def modified_toeplitz_hash_batched(blocks, stream=None):
    """blocks: sequence of (key, n, v, m, out) tuples (v: n-1 bits); returns the outs."""
    arr = _blocks(blocks, lambda n, m: (n + 62) >> 6)
    _check(lib().pa_modified_toeplitz_hash_batched(arr, len(blocks), _stream_handle(stream)))
    return [b[4] for b in blocks]


class BatchGraph:
    """Captured batched call over fixed buffers (pa_graph_*); launch() replays it."""

    def __init__(self, blocks, modified: bool = False):
        self._modified = bool(modified)
        arr = self._arr(blocks)
        h = ctypes.c_void_p()
        _check(lib().pa_graph_create(arr, len(blocks), 1 if modified else 0, ctypes.byref(h)))
        self._h = h
        self._keep = list(blocks)   # the buffers the graph reads and writes

    def _arr(self, blocks):
        if self._modified:
            return _blocks(blocks, lambda n, m: (n + 62) >> 6)
        return _blocks(blocks, lambda n, m: (n + m + 62) >> 6)

    def update(self, blocks, stream=None):
        """Point the graph at other buffers (same length groups)."""
        _check(lib().pa_graph_update(self._h, self._arr(blocks), len(blocks), _stream_handle(stream)))
        self._keep = list(blocks)

    def launch(self, stream=None):
        _check(lib().pa_graph_launch(self._h, _stream_handle(stream)))

    @property
    def block_count(self) -> int:
        return int(lib().pa_graph_block_count(self._h))

    def destroy(self):
        if self._h:
            _check(lib().pa_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fft_pair_transform_len(n: int, m: int) -> int:
    return int(lib().pa_fft_pair_transform_len(int(n), int(m)))


def toeplitz_hash_pair_fft(key_a, key_b, n: int, seed, m: int, out_a=None, out_b=None, guard: float = 0.25,
                           stream=None):
    """Two keys with one seed through one FP64 complex FFT; returns
    (out_a, out_b, max_error, fell_back).  Blocks until the error is known."""
    import torch
    if out_a is None:
        out_a = torch.empty(max(words(m), 1), dtype=torch.int64, device=key_a.device)
    if out_b is None:
        out_b = torch.empty(max(words(m), 1), dtype=torch.int64, device=key_a.device)
    err = ctypes.c_double()
    fb = ctypes.c_int()
    _check(lib().pa_toeplitz_hash_pair_fft(_ptr(key_a, words(n), "key_a"), _ptr(key_b, words(n), "key_b"), int(n),
                                           _ptr(seed, words(n + m - 1), "seed"), int(m), _ptr(out_a, words(m), "out_a"),
                                           _ptr(out_b, words(m), "out_b"), float(guard), _stream_handle(stream),
                                           ctypes.byref(err), ctypes.byref(fb)))
    return out_a, out_b, err.value, bool(fb.value)


def alu_probe(stream=None) -> dict:
    """Measured fp64 FMA rate (T/s) and exact modular-product rate (G/s)."""
    f, m = ctypes.c_double(), ctypes.c_double()
    _check(lib().pa_alu_probe(_stream_handle(stream), ctypes.byref(f), ctypes.byref(m)))
    return {"fma_Tops": f.value, "mulmod_Gops": m.value}


def launch_probe(workgroups: int, threads: int, reps: int = 200, stream=None) -> float:
    """Microseconds per back-to-back launch of an empty kernel of this shape."""
    us = ctypes.c_double()
    _check(lib().pa_launch_probe(_stream_handle(stream), int(workgroups), int(threads), int(reps), ctypes.byref(us)))
    return us.value


def phase_probe(stream=None) -> dict:
    """Three dependent phases as three launches and as one cooperative
    launch with grid barriers; per-tile release cost (see include/pa.h)."""
    r = PhaseProbeResult()
    _check(lib().pa_phase_probe(_stream_handle(stream), ctypes.byref(r)))
    return {f: (getattr(r, f) if isinstance(getattr(r, f), float) else int(getattr(r, f))) for f, _ in r._fields_}


def final_key_length(n: int, t: int, s: int) -> int:
    """Output length r = n - t - s of the hash (0 if t + s >= n)."""
    return int(lib().pa_final_key_length(int(n), int(t), int(s)))


class Plan:
    """Seed spectrum resident on the device (pa_plan_*)."""

    def __init__(self, seed, seed_len_bits: int, transform_len: int = 0, stream=None):
        h = ctypes.c_void_p()
        _check(lib().pa_plan_create(_ptr(seed, words(seed_len_bits), "seed"), int(seed_len_bits),
                                    int(transform_len), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.seed_len_bits = int(seed_len_bits)

    @property
    def transform_len(self) -> int:
        return int(lib().pa_plan_transform_len(self._h))

    def hash(self, key, n: int, m: int, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(max(words(m), 1), dtype=torch.int64, device=key.device)
        _check(lib().pa_plan_hash(self._h, _ptr(key, words(n), "key"), int(n), int(m),
                                  _ptr(out, words(m), "out"), _stream_handle(stream)))
        return out

    def spectrum(self, out=None, stream=None):
        """The resident seed spectrum (int32 tensor of transform_len values,
        reduced residues in transform order)."""
        import torch
        L = self.transform_len
        if out is None:
            out = torch.empty(L, dtype=torch.int32, device="cuda")
        if not out.is_cuda or out.dtype != torch.int32 or not out.is_contiguous() or out.numel() < L:
            raise ValueError("out must be a contiguous int32 device tensor of transform_len values")
        _check(lib().pa_plan_spectrum(self._h, out.data_ptr(), _stream_handle(stream)))
        return out

    def destroy(self):
        if self._h:
            _check(lib().pa_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()
        return False


EXEC_GPU = 0
EXEC_SIMULATED = 1


class Server:
    """Continuous-batching serving loop (pa_server_*).

    Pointers are device addresses (ints) or torch CUDA tensors; the caller
    keeps them alive until the request completes.  With
    executor=EXEC_SIMULATED nothing touches the device.
    """

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 256, max_queue: int = 1 << 20,
                 streams: int = 4, executor: int = EXEC_GPU, sim_bits_per_us: float = 1e4, sim_fail_every: int = 0):
        cfg = ServerConfig(int(hbm_budget_bytes), int(max_inflight), int(max_queue), int(streams), int(executor),
                           float(sim_bits_per_us), int(sim_fail_every))
        h = ctypes.c_void_p()
        _check(lib().pa_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def _addr(x, nwords, what):
        if isinstance(x, int):
            return x
        return _ptr(x, nwords, what)

    def register_seed(self, seed, seed_len_bits: int) -> int:
        sid = ctypes.c_uint32()
        _check(lib().pa_server_register_seed(self._h, self._addr(seed, words(seed_len_bits), "seed"),
                                             int(seed_len_bits), ctypes.byref(sid)))
        return sid.value

    def submit(self, seed_id: int, key, n: int, m: int, out) -> int:
        t = ctypes.c_uint64()
        _check(lib().pa_server_submit(self._h, int(seed_id), self._addr(key, words(n), "key"), int(n), int(m),
                                      self._addr(out, words(m), "out"), ctypes.byref(t)))
        return t.value

    def cancel(self, ticket: int):
        """Cancels a request that is still queued (raises PAError with
        PA_ERR_BUSY if it has already been admitted)."""
        _check(lib().pa_server_cancel(self._h, int(ticket)))

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _check(lib().pa_server_poll(self._h, int(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> float:
        lat = ctypes.c_double()
        _check(lib().pa_server_wait(self._h, int(ticket), ctypes.byref(lat)))
        return lat.value

    def latency_us(self, ticket: int) -> float:
        lat = ctypes.c_double()
        _check(lib().pa_server_latency(self._h, int(ticket), ctypes.byref(lat)))
        return lat.value

    def drain(self):
        _check(lib().pa_server_drain(self._h))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().pa_server_stats_get(self._h, ctypes.byref(st)))
        return {f: int(getattr(st, f)) for f, _ in st._fields_}

    def close(self):
        if self._h:
            _check(lib().pa_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False
