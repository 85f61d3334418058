"""Row kernels compiled for fixed row-transform shapes, against the oracle.

Each fixed shape (the row transform of the default geometry of the lengths
2^18 .. 27 * 2^19) runs here at the smallest length that uses it, on the
plain path (seed and key rows in one kernel), the plan path (key row against
a resident spectrum, after the spectrum-building mode of the same kernel)
and a batched call, and must give the oracle's bits (Sec. 2.3 Eq. (4): the
product of the Toeplitz matrix and the key).  The same length under a
row split that no fixed kernel covers runs the general kernel and must
give the same bits.
"""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def shape_lengths():
    """Smallest supported length per fixed row shape (default geometry)."""
    first = {}
    for L in pa.supported_lengths():
        d = pa.plan_info(L)
        if d["row_shape"] and d["row_shape"] not in first:
            first[d["row_shape"]] = L
    return sorted(first.items())


SHAPES = shape_lengths()


def block_for(L):
    """(n, m) whose transform length is L: m = n/4 up to about 1.2e6 bits,
    a 20,000-bit window beyond (the oracle's cost grows with n * m)."""
    small = L <= 3 * 2**19
    n = (L - 256) * 4 // 5 if small else L - 20_000 - 256
    m = n // 4 if small else 20_000
    assert pa.transform_len(n, m) == L, (L, n, m)
    return n, m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t, m):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)[: wl.words(m)]


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()


def test_every_fixed_shape_is_exercised():
    assert len(SHAPES) >= 10
    for sh, L in SHAPES:
        assert 2**18 <= L <= 27 * 2**19, (sh, L)


@pytest.mark.parametrize("sh,L", SHAPES, ids=[f"shape{s}_L{L}" for s, L in SHAPES])
def test_fixed_row_shape_matches_oracle(sh, L):
    n, m = block_for(L)
    print("row shape %d: L=%d C=%d n=%d m=%d" % (sh, L, pa.plan_info(L)["cols"], n, m), flush=True)
    key, seed = wl.key_and_seed(60 + sh, n, m, 0)
    want = oracle.toeplitz_hash(key, n, seed, m)
    dk, ds = dev(key), dev(seed)
    # plain path
    assert np.array_equal(host(pa.toeplitz_hash(dk, n, ds, m), m), want), "plain"
    # plan path: the spectrum built by the row kernel's seed mode, then the key
    with pa.Plan(ds, n + m - 1, transform_len=L) as plan:
        assert np.array_equal(host(plan.hash(dk, n, m), m), want), "plan"
    # batched: this block and a second one of the same length
    key2, seed2 = wl.key_and_seed(60 + sh, n, m, 1)
    want2 = oracle.toeplitz_hash(key2, n, seed2, m)
    outs = [torch.zeros(wl.words(m), dtype=torch.int64, device="cuda") for _ in range(2)]
    pa.toeplitz_hash_batched([(dk, n, ds, m, outs[0]), (dev(key2), n, dev(seed2), m, outs[1])])
    assert np.array_equal(host(outs[0], m), want), "batched 0"
    assert np.array_equal(host(outs[1], m), want2), "batched 1"


def test_general_kernel_at_a_fixed_shape_length():
    # L = 3 * 2^19 under R = 128 has rows of 12,288 values: no fixed kernel
    L = 3 * 2**19
    assert pa.plan_info(L)["row_shape"] != 0 and pa.plan_info(L, 7)["row_shape"] == 0
    n, m = block_for(L)
    key, seed = wl.key_and_seed(71, n, m, 0)
    want = oracle.toeplitz_hash(key, n, seed, m)
    dk, ds = dev(key), dev(seed)
    a0, w0 = pa.tune_get(L, 0)
    try:
        pa.tune_set(L, 0, 7, 0)
        assert np.array_equal(host(pa.toeplitz_hash(dk, n, ds, m), m), want)
    finally:
        pa.tune_set(L, 0, 0, 0)
    assert pa.tune_get(L, 0) == (a0, w0)
    assert np.array_equal(host(pa.toeplitz_hash(dk, n, ds, m), m), want)
