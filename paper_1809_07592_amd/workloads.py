"""Seeded synthetic inputs for Toeplitz-hash privacy amplification.

This module only draws random numbers and describes workload shapes; it
contains none of the hash's arithmetic.  Both the GPU path's tests/benchmark
and the CPU oracle take their inputs from here.

Raw QKD keys are not available, so i.i.d. Bernoulli(0.5) bits stand in for
the reconciled key and for the Toeplitz seed (the paper's "random sequence",
Sec. 2.2).  Bits are little-endian packed uint64: bit k in word k >> 6,
position k & 63.  Every generator is a PCG64 stream keyed by
SeedSequence([config_id, role, index]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ROLE_KEY = 1
ROLE_SEED = 2
ROLE_SIZES = 3
ROLE_ARRIVALS = 4
ROLE_GARBAGE = 5


def rng(config_id: int, role: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(config_id), int(role), int(index)])))


def words(bits: int) -> int:
    return (int(bits) + 63) // 64


def random_bits(nbits: int, gen: np.random.Generator, garbage_tail: bool = False) -> np.ndarray:
    """ceil(nbits/64) uniform words; bits >= nbits are zero unless garbage_tail."""
    nw = max(words(nbits), 1)
    a = gen.integers(0, 2**64 - 1, size=nw, dtype=np.uint64, endpoint=True)
    if nbits == 0:
        a[:] = 0
        return a
    if nbits % 64 and not garbage_tail:
        a[-1] &= np.uint64((1 << (nbits % 64)) - 1)
    return a


def key_and_seed(config_id: int, n: int, m: int, index: int = 0, garbage_tail: bool = False):
    """(key, seed) for one block: n key bits, n+m-1 seed bits."""
    key = random_bits(n, rng(config_id, ROLE_KEY, index), garbage_tail)
    seed = random_bits(n + m - 1, rng(config_id, ROLE_SEED, index), garbage_tail)
    return key, seed


@dataclass(frozen=True)
class BlockShape:
    n: int
    m: int


# Single-block configurations (key bits n, output bits m).
CONFIG_SMALL = BlockShape(262_144, 65_536)            # oracle-sized, several tiles + ragged tail
CONFIG_FINITE_SIZE = BlockShape(1_000_000, 250_000)   # the paper's n >= 10^6 finite-size block, ratio 0.25
CONFIG_LARGE = BlockShape(12_800_000, 1_280_000)      # 12.8M-bit block, ratio 0.1


def batched_shapes(count: int = 256, config_id: int = 4):
    """n log-uniform in [2^18, 2^22], m/n uniform in [0.05, 0.5]."""
    g = rng(config_id, ROLE_SIZES, 0)
    out = []
    for _ in range(count):
        n = int(round(2.0 ** g.uniform(18.0, 22.0)))
        m = max(1, int(round(n * g.uniform(0.05, 0.5))))
        out.append(BlockShape(n, min(m, n)))
    return out


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n: int
    m: int
    seed_id: int


def serving_requests(count: int = 10_000, rate_per_s: float = 1000.0, n_seeds: int = 16, config_id: int = 5):
    """Poisson arrivals; n log-uniform in [1e5, 1e7]; m/n uniform in [0.1, 0.5]."""
    gs = rng(config_id, ROLE_SIZES, 0)
    ga = rng(config_id, ROLE_ARRIVALS, 0)
    gaps = ga.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    reqs = []
    for i in range(count):
        n = int(round(10.0 ** gs.uniform(5.0, 7.0)))
        m = max(1, min(n, int(round(n * gs.uniform(0.1, 0.5)))))
        sid = int(gs.integers(0, n_seeds))
        reqs.append(Request(i, float(t[i]), n, m, sid))
    return reqs


def serving_mean_n() -> float:
    """E[n] for n = 10^U(5,7): (1e7 - 1e5) / (2 ln 10)."""
    return (1e7 - 1e5) / (2.0 * math.log(10.0))
