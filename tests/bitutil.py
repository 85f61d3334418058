"""Small helpers for tests: packed uint64 <-> 0/1 arrays and Python ints.

Little-endian packing: bit k lives in word k >> 6 at position k & 63.
"""
import numpy as np


def unpack(words: np.ndarray, nbits: int) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint64)
    b = np.unpackbits(w.view(np.uint8), bitorder="little")
    return b[:nbits].astype(np.uint8)


def pack(bits) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.uint8)
    nw = max((bits.size + 63) // 64, 1)
    padded = np.zeros(nw * 64, dtype=np.uint8)
    padded[: bits.size] = bits
    return np.packbits(padded, bitorder="little").view(np.uint64).copy()


def to_int(bits) -> int:
    """Bit string -> Python int with bit k = bits[k]."""
    bits = np.asarray(bits, dtype=np.uint8)
    if bits.size == 0:
        return 0
    return int.from_bytes(np.packbits(bits, bitorder="little").tobytes(), "little")


def from_int(v: int, nbits: int) -> np.ndarray:
    v &= (1 << nbits) - 1
    nbytes = (nbits + 7) // 8
    raw = np.frombuffer(v.to_bytes(max(nbytes, 1), "little"), dtype=np.uint8)
    return np.unpackbits(raw, bitorder="little")[:nbits].astype(np.uint8)


def tail_is_zero(words: np.ndarray, nbits: int) -> bool:
    w = np.asarray(words, dtype=np.uint64)
    nw = (nbits + 63) // 64
    if nbits % 64:
        if int(w[nw - 1]) >> (nbits % 64):
            return False
    return bool(np.all(w[nw:] == 0))
