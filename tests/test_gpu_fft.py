"""FP64 complex-FFT pair form on the GPU (the paper's float route, two real
sequences per complex transform): both outputs equal the CPU oracle bit for
bit, the reported rounding error stays far below the 1/4 margin up to the
largest length (2^24), and a guard the error reaches switches both keys to
the exact number-theoretic path."""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t, m):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)[: wl.words(m)]


@pytest.fixture(autouse=True, scope="module")
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    yield


def pair(cfg, n, m, idx=0):
    ka = wl.random_bits(n, wl.rng(cfg, wl.ROLE_KEY, 2 * idx))
    kb = wl.random_bits(n, wl.rng(cfg, wl.ROLE_KEY, 2 * idx + 1))
    s = wl.random_bits(n + m - 1, wl.rng(cfg, wl.ROLE_SEED, idx))
    return ka, kb, s


@pytest.mark.parametrize("n,m", [(1, 1), (2, 1), (64, 64), (65, 1), (1000, 500), (4097, 2048), (100_003, 31_337),
                                 (262_144, 65_536), (300_000, 27_001)])
def test_pair_matches_oracle(n, m):
    ka, kb, s = pair(70, n, m, n)
    ya, yb, err, fb = pa.toeplitz_hash_pair_fft(dev(ka), dev(kb), n, dev(s), m)
    assert not fb and 0.0 <= err < 1e-6
    assert np.array_equal(host(ya, m), oracle.toeplitz_hash(ka, n, s, m))
    assert np.array_equal(host(yb, m), oracle.toeplitz_hash(kb, n, s, m))


def test_finite_size_block():
    n, m = 1_000_000, 250_000
    ka, kb, s = pair(71, n, m)
    ya, yb, err, fb = pa.toeplitz_hash_pair_fft(dev(ka), dev(kb), n, dev(s), m)
    print("n=1e6 max rounding error %.3g" % err)
    assert not fb and err < 1e-3
    assert np.array_equal(host(ya, m), oracle.toeplitz_hash(ka, n, s, m))
    assert np.array_equal(host(yb, m), oracle.toeplitz_hash(kb, n, s, m))


def test_largest_length_sampled():
    n, m = 12_800_000, 1_280_000
    assert pa.fft_pair_transform_len(n, m) == 2**24
    ka, kb, s = pair(72, n, m)
    ya, yb, err, fb = pa.toeplitz_hash_pair_fft(dev(ka), dev(kb), n, dev(s), m)
    print("n=12.8e6 max rounding error %.3g" % err)
    assert not fb and err < 0.25
    idx = np.sort(np.random.default_rng(73).choice(m, 300, replace=False)).astype(np.uint64)
    for k, y in ((ka, ya), (kb, yb)):
        w = host(y, m)
        got = ((w[idx >> np.uint64(6)] >> (idx & np.uint64(63))) & np.uint64(1)).astype(np.uint8)
        assert np.array_equal(got, oracle.toeplitz_bits(k, n, s, m, idx))


def test_all_ones_keys_extreme_values():
    n, m = 200_000, 50_000
    ka = wl.random_bits(n, wl.rng(74, wl.ROLE_KEY, 0))
    kb = np.full(wl.words(n), np.uint64(2**64 - 1), dtype=np.uint64)
    kb[-1] &= np.uint64((1 << (n % 64)) - 1) if n % 64 else np.uint64(2**64 - 1)
    s = np.full(wl.words(n + m - 1), np.uint64(2**64 - 1), dtype=np.uint64)
    ya, yb, err, fb = pa.toeplitz_hash_pair_fft(dev(ka), dev(kb), n, dev(s), m)
    assert not fb
    assert np.array_equal(host(ya, m), oracle.toeplitz_hash(ka, n, s, m))
    assert np.array_equal(host(yb, m), oracle.toeplitz_hash(kb, n, s, m))


def test_guard_falls_back_to_exact_path():
    n, m = 50_000, 20_000
    ka, kb, s = pair(75, n, m)
    ya, yb, err, fb = pa.toeplitz_hash_pair_fft(dev(ka), dev(kb), n, dev(s), m, guard=0.0)
    assert fb and err >= 0.0
    assert np.array_equal(host(ya, m), oracle.toeplitz_hash(ka, n, s, m))
    assert np.array_equal(host(yb, m), oracle.toeplitz_hash(kb, n, s, m))
