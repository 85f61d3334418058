"""Pins for the CPU oracle, independent of its own code (no GPU).

The paper (Sec. 2.2) defines the hash as the product of an m x n Toeplitz
matrix over GF(2) with the key; it prints no numeric example, so the oracle
is pinned by mathematics instead:
  * brute force with the explicit matrix on tiny inputs (exhaustive where
    feasible),
  * closed forms for unit keys/seeds and all-ones keys/seeds,
  * bilinearity and the diagonal-constant shift structure of T,
  * the prefix property (extra seed bits never matter),
  * a textbook reduction: y is the middle of the polynomial product
    s(z) x(z) over GF(2) -- checked by a carry-less Python-int product and by
    Kronecker substitution into one big-integer multiplication.
Each is chosen so that a plausible mistake (Hankel instead of Toeplitz,
reversed output, off-by-one window, swapped operands, dropped tail word)
fails at least one of them.
"""

import numpy as np
import pytest

from bitutil import from_int, pack, tail_is_zero, to_int, unpack
from paper_1809_07592_amd import workloads as wl


def explicit_T(s_bits, n, m):
    """T[i][j] = s[i - j + n - 1] (first row s[n-1..0], first column s[n-1..n+m-2])."""
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    return np.asarray(s_bits, dtype=np.int64)[i - j + n - 1]


def brute(x_bits, s_bits, n, m):
    return (explicit_T(s_bits, n, m) @ np.asarray(x_bits, dtype=np.int64)) % 2


def run(oracle, x_bits, s_bits, n, m):
    out = oracle.toeplitz_hash(pack(x_bits), n, pack(s_bits), m)
    assert tail_is_zero(out, m)
    return unpack(out, m)


def test_matrix_is_toeplitz_with_stated_corners():
    s = np.arange(10)
    T = explicit_T(s, 6, 5)
    assert list(T[0]) == [5, 4, 3, 2, 1, 0]          # first row s[n-1], ..., s[0]
    assert list(T[:, 0]) == [5, 6, 7, 8, 9]          # first column s[n-1], ..., s[n+m-2]
    assert all(T[i + 1, j + 1] == T[i, j] for i in range(4) for j in range(5))


def test_exhaustive_tiny(oracle):
    # every key and every seed for n+m-1 <= 7
    for n in range(1, 6):
        for m in range(1, n + 1):
            L = n + m - 1
            if L > 7:
                continue
            for sv in range(1 << L):
                s = [(sv >> k) & 1 for k in range(L)]
                for xv in range(1 << n):
                    x = [(xv >> k) & 1 for k in range(n)]
                    assert list(run(oracle, x, s, n, m)) == list(brute(x, s, n, m)), (n, m, sv, xv)


def test_brute_force_random_small(oracle):
    g = np.random.default_rng(7)
    for n in list(range(1, 140)) + [191, 192, 193, 255, 256, 257]:
        for m in sorted({1, min(2, n), n // 3 or 1, n // 2 or 1, n - 1 or 1, n}):
            x = g.integers(0, 2, n)
            s = g.integers(0, 2, n + m - 1)
            assert np.array_equal(run(oracle, x, s, n, m), brute(x, s, n, m)), (n, m)


def test_unit_key_gives_a_column(oracle):
    # x = e_j  =>  y_i = T[i][j] = s[i - j + n - 1]
    g = np.random.default_rng(11)
    n, m = 300, 170
    s = g.integers(0, 2, n + m - 1)
    for j in [0, 1, 63, 64, 65, 150, n - 1]:
        x = np.zeros(n, np.uint8)
        x[j] = 1
        expect = [s[i - j + n - 1] for i in range(m)]
        assert list(run(oracle, x, s, n, m)) == expect


def test_unit_seed_shifts_the_key(oracle):
    # s = e_k  =>  y_i = x[i + n - 1 - k] if 0 <= i+n-1-k < n else 0
    g = np.random.default_rng(12)
    n, m = 257, 100
    x = g.integers(0, 2, n)
    for k in [0, 5, 64, n - 1, n + m - 2, 200]:
        s = np.zeros(n + m - 1, np.uint8)
        s[k] = 1
        expect = [x[i + n - 1 - k] if 0 <= i + n - 1 - k < n else 0 for i in range(m)]
        assert list(run(oracle, x, s, n, m)) == expect


def test_all_ones_key_is_window_parity(oracle):
    # x = 1^n  =>  y_i = XOR_{t<n} s[i+t] = P[i+n] ^ P[i] (P = prefix XOR of s)
    g = np.random.default_rng(13)
    n, m = 1000, 333
    s = g.integers(0, 2, n + m - 1)
    P = np.concatenate([[0], np.bitwise_xor.accumulate(s)])
    expect = [P[i + n] ^ P[i] for i in range(m)]
    assert list(run(oracle, np.ones(n, np.uint8), s, n, m)) == expect


def test_all_ones_seed_gives_key_parity(oracle):
    g = np.random.default_rng(14)
    n, m = 777, 300
    x = g.integers(0, 2, n)
    y = run(oracle, x, np.ones(n + m - 1, np.uint8), n, m)
    assert set(y.tolist()) == {int(x.sum() % 2)}


def test_bilinear(oracle):
    g = np.random.default_rng(15)
    n, m = 2000, 640
    x1, x2 = g.integers(0, 2, n), g.integers(0, 2, n)
    s1, s2 = g.integers(0, 2, n + m - 1), g.integers(0, 2, n + m - 1)
    assert np.array_equal(run(oracle, x1 ^ x2, s1, n, m), run(oracle, x1, s1, n, m) ^ run(oracle, x2, s1, n, m))
    assert np.array_equal(run(oracle, x1, s1 ^ s2, n, m), run(oracle, x1, s1, n, m) ^ run(oracle, x1, s2, n, m))


def test_key_shift_moves_output_down(oracle):
    # T[i+1][j+1] = T[i][j]: with x_{n-1} = 0 and x' = (0, x_0..x_{n-2}), y'_{i+1} = y_i
    g = np.random.default_rng(16)
    n, m = 1500, 400
    x = g.integers(0, 2, n)
    x[n - 1] = 0
    s = g.integers(0, 2, n + m - 1)
    xs = np.concatenate([[0], x[:-1]])
    y, ys = run(oracle, x, s, n, m), run(oracle, xs, s, n, m)
    assert np.array_equal(ys[1:], y[:-1])


def test_seed_shift_moves_output_up(oracle):
    # s' = s[1:] || b  =>  y'_i = y_{i+1}
    g = np.random.default_rng(17)
    n, m = 1300, 500
    x = g.integers(0, 2, n)
    s = g.integers(0, 2, n + m - 1)
    s2 = np.concatenate([s[1:], [1]])
    y, y2 = run(oracle, x, s, n, m), run(oracle, x, s2, n, m)
    assert np.array_equal(y2[:-1], y[1:])


def test_prefix_property_and_padding_garbage(oracle):
    # extra seed bits and garbage padding bits never change y; out tail is zero
    n, m = 1000, 237
    key, seed = wl.key_and_seed(99, n, m, 0, garbage_tail=False)
    ref = oracle.toeplitz_hash(key, n, seed, m)
    gkey, gseed = wl.key_and_seed(99, n, m, 0, garbage_tail=True)
    assert np.array_equal(gkey[:-1], key[:-1]) and gkey[-1] != key[-1]
    longer = np.concatenate([gseed, wl.random_bits(5000, wl.rng(99, wl.ROLE_GARBAGE, 1))])
    for k, s in [(key, seed), (gkey, gseed), (gkey, longer)]:
        out = oracle.toeplitz_hash(k, n, s, m)
        assert np.array_equal(out, ref)
        assert tail_is_zero(out, m)


def gf2_mul(a: int, b: int) -> int:
    """Carry-less product of two GF(2)[z] polynomials held in Python ints."""
    r = 0
    while b:
        low = b & -b
        r ^= a << (low.bit_length() - 1)
        b ^= low
    return r


def test_middle_product_over_gf2(oracle):
    # y_i is coefficient n-1+i of s(z) x(z) in GF(2)[z]
    g = np.random.default_rng(18)
    for n, m in [(64, 64), (100, 1), (1000, 300), (4096, 1024), (3001, 2999)]:
        x = g.integers(0, 2, n)
        s = g.integers(0, 2, n + m - 1)
        prod = gf2_mul(to_int(s), to_int(x))
        expect = from_int(prod >> (n - 1), m)
        assert np.array_equal(run(oracle, x, s, n, m), expect), (n, m)


def test_kronecker_integer_product(oracle):
    # c = s * x as integer sequences via one big-integer product with g-bit
    # digits (g > log2 n so no carries cross digits); y_i = c[n-1+i] mod 2.
    n, m = 65_536, 16_384
    key, seed = wl.key_and_seed(1, n, m, 3)
    xb, sb = unpack(key, n), unpack(seed, n + m - 1)
    gbits = n.bit_length() + 1

    def spread(bits):
        # place bit k at bit position gbits*k of one big integer
        positions = np.flatnonzero(bits).astype(np.int64) * gbits
        buf = np.zeros((int(positions.max()) // 8 + 1) if positions.size else 1, dtype=np.uint8)
        np.bitwise_or.at(buf, positions // 8, (1 << (positions % 8)).astype(np.uint8))
        return int.from_bytes(buf.tobytes(), "little")

    C = spread(sb) * spread(xb)
    mask = (1 << gbits) - 1
    expect = np.array([((C >> (gbits * (n - 1 + i))) & mask) & 1 for i in range(m)], dtype=np.uint8)
    got = unpack(oracle.toeplitz_hash(key, n, seed, m), m)
    assert np.array_equal(got, expect)


def test_bits_sampler_matches_full(oracle):
    n, m = 20_000, 7_001
    key, seed = wl.key_and_seed(2, n, m, 0)
    full = unpack(oracle.toeplitz_hash(key, n, seed, m), m)
    idx = np.array([0, 1, 63, 64, 65, 4000, m - 2, m - 1], dtype=np.uint64)
    assert np.array_equal(oracle.toeplitz_bits(key, n, seed, m, idx), full[idx.astype(np.int64)])


def explicit_modified(x_bits, v_bits, n, m):
    """S = [I_m | V], V[i][j] = v[i - j + (n-m) - 1] (Eq. (2)-(3), reading in DESIGN)."""
    nt = n - m
    i = np.arange(m)[:, None]
    j = np.arange(nt)[None, :]
    V = np.asarray(v_bits, dtype=np.int64)[i - j + nt - 1]
    S = np.concatenate([np.eye(m, dtype=np.int64), V], axis=1)
    return (S @ np.asarray(x_bits, dtype=np.int64)) % 2


def test_modified_toeplitz_brute(oracle):
    g = np.random.default_rng(19)
    for n in [2, 3, 5, 17, 64, 65, 130, 301]:
        for m in sorted({1, n // 2 or 1, n - 1}):
            if not 1 <= m < n:
                continue
            x = g.integers(0, 2, n)
            v = g.integers(0, 2, n - 1)
            out = oracle.modified_toeplitz_hash(pack(x), n, pack(v), m)
            assert tail_is_zero(out, m)
            assert np.array_equal(unpack(out, m), explicit_modified(x, v, n, m)), (n, m)


def test_modified_reduces_to_identity_plus_plain(oracle):
    # y = x[0:m] xor Toeplitz(v) x[m:n]: with x[m:n] = 0 the output is x[0:m]
    g = np.random.default_rng(20)
    n, m = 900, 300
    x = g.integers(0, 2, n)
    x[m:] = 0
    v = g.integers(0, 2, n - 1)
    assert np.array_equal(unpack(oracle.modified_toeplitz_hash(pack(x), n, pack(v), m), m), x[:m])


def test_rejects_bad_shapes(oracle):
    k = np.zeros(4, np.uint64)
    for n, m in [(0, 1), (10, 0), (10, 11)]:
        with pytest.raises(ValueError):
            oracle.toeplitz_hash(k, n, np.zeros(8, np.uint64), m)
