"""CPU oracle for Toeplitz-hash privacy amplification.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does and
shares no code with it.  See ``toeplitz_oracle.c`` for the definition it
computes (paper Sec. 2.1-2.2: y = T x over GF(2), T[i][j] = s[i-j+n-1]).

Arrays are numpy ``uint64`` little-endian packed bit strings (bit k in word
k >> 6, position k & 63).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "toeplitz_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_NATIVE_PATH = os.path.join(_HERE, "liboracle_native.so")
_lib = None
_lib_path = None


def build(force: bool = False, native: bool = False) -> str:
    """Compile the oracle with gcc/OpenMP.  The default build is portable
    x86-64-v3 code (it may be built on one machine and run on another);
    native=True builds liboracle_native.so for the CPU it is compiled on
    (-march=native), for timing the oracle on the machine that runs it."""
    path = _NATIVE_PATH if native else _LIB_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=native" if native else "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC",
               "-std=c99", "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


def select_native() -> str:
    """Compile for the CPU of this machine (always, since a build from
    another machine may use instructions this one lacks) and switch every
    later call to that build of the same source."""
    global _lib, _lib_path
    path = build(force=True, native=True)
    _lib, _lib_path = None, path
    _load()
    return path


def _load():
    global _lib
    if _lib is None:
        path = _lib_path or _LIB_PATH
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_toeplitz_hash.argtypes = [u64p, ctypes.c_uint64, u64p, ctypes.c_uint64, u64p, ctypes.c_int]
        lib.oracle_toeplitz_hash.restype = ctypes.c_int
        lib.oracle_toeplitz_bits.argtypes = [u64p, ctypes.c_uint64, u64p, ctypes.c_uint64, u64p,
                                             ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int]
        lib.oracle_toeplitz_bits.restype = ctypes.c_int
        lib.oracle_modified_toeplitz_hash.argtypes = [u64p, ctypes.c_uint64, u64p, ctypes.c_uint64, u64p, ctypes.c_int]
        lib.oracle_modified_toeplitz_hash.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _words(bits: int) -> int:
    return (bits + 63) // 64


def _as_u64(a: np.ndarray, min_words: int, what: str) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if a.size < min_words:
        raise ValueError("%s has %d words, needs %d" % (what, a.size, min_words))
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def toeplitz_hash(key: np.ndarray, n: int, seed: np.ndarray, m: int, threads: int = 0) -> np.ndarray:
    """y = T x over GF(2) for the m x n Toeplitz matrix of the n+m-1 seed bits."""
    key = _as_u64(key, _words(n), "key")
    seed = _as_u64(seed, _words(n + m - 1), "seed")
    out = np.zeros(max(_words(m), 1), dtype=np.uint64)
    rc = _load().oracle_toeplitz_hash(_p(key), n, _p(seed), m, _p(out), int(threads))
    if rc != 0:
        raise ValueError("oracle_toeplitz_hash failed with code %d (n=%d, m=%d)" % (rc, n, m))
    return out


def toeplitz_bits(key: np.ndarray, n: int, seed: np.ndarray, m: int, idx, threads: int = 0) -> np.ndarray:
    """Output bits y_i for the requested indices i (uint8 array of 0/1)."""
    key = _as_u64(key, _words(n), "key")
    seed = _as_u64(seed, _words(n + m - 1), "seed")
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    bits = np.zeros(max(idx.size, 1), dtype=np.uint8)
    rc = _load().oracle_toeplitz_bits(_p(key), n, _p(seed), m, _p(idx), idx.size,
                                      bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(threads))
    if rc != 0:
        raise ValueError("oracle_toeplitz_bits failed with code %d" % rc)
    return bits[: idx.size]


def modified_toeplitz_hash(key: np.ndarray, n: int, vbits: np.ndarray, m: int, threads: int = 0) -> np.ndarray:
    """y = x[0:m] XOR V x[m:n] (paper Eq. (2)-(3)), V described by n-1 bits."""
    key = _as_u64(key, _words(n), "key")
    vbits = _as_u64(vbits, _words(n - 1), "vbits")
    out = np.zeros(max(_words(m), 1), dtype=np.uint64)
    rc = _load().oracle_modified_toeplitz_hash(_p(key), n, _p(vbits), m, _p(out), int(threads))
    if rc != 0:
        raise ValueError("oracle_modified_toeplitz_hash failed with code %d (n=%d, m=%d)" % (rc, n, m))
    return out
