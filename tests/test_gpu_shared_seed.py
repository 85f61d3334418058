"""Batched calls whose blocks share a seed, against the CPU oracle.

In the lanes form, blocks of one transform length that pass the same seed
(device pointer and bit count) run the key path against that seed's
spectrum, built once per call, instead of each transforming the seed.  The
result must not change: every block equals the oracle's product of its own
Toeplitz matrix and key (Sec. 2.3 Eq. (4)), in a batch that mixes shared
and own seeds, seeds shared by blocks of different (n, m) with the same
seed length, one pointer used with two seed lengths (two spectra), the
modified Toeplitz form, and captured graphs and their updates.
"""
import os

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


def out_for(m):
    return torch.full((wl.words(m),), -1, dtype=torch.int64, device="cuda")


@pytest.fixture(autouse=True)
def _lanes_form():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    old = os.environ.pop("PA_BATCH_FORM", None)
    yield
    if old is not None:
        os.environ["PA_BATCH_FORM"] = old


def mixed_batch():
    """(key, seed, n, m) items and the seed tensors they use: 1e6-bit blocks
    sharing seed A (12 blocks), 2 on seed B with (n, m) and (n + 5, m - 5),
    3 with their own seeds, and seed A's pointer with a shorter length."""
    n, m = 1_000_000, 250_000
    seed_a = wl.random_bits(n + m - 1, wl.rng(120, wl.ROLE_SEED, 0))
    seed_b = wl.random_bits(n + m - 1, wl.rng(120, wl.ROLE_SEED, 1))
    d_a, d_b = dev(seed_a), dev(seed_b)
    items = []
    for i in range(12):
        items.append((wl.random_bits(n, wl.rng(120, wl.ROLE_KEY, i)), seed_a, d_a, n, m))
    items.append((wl.random_bits(n, wl.rng(121, wl.ROLE_KEY, 0)), seed_b, d_b, n, m))
    items.append((wl.random_bits(n + 5, wl.rng(121, wl.ROLE_KEY, 1)), seed_b, d_b, n + 5, m - 5))
    for i in range(3):
        key, seed = wl.key_and_seed(122, n, m, i)
        items.append((key, seed, dev(seed), n, m))
    # seed A's first 1,000,000 + 200,000 - 1 bits: another spectrum, same pointer
    n2, m2 = 1_000_000, 200_000
    for i in range(2):
        items.append((wl.random_bits(n2, wl.rng(123, wl.ROLE_KEY, i)), seed_a[: wl.words(n2 + m2 - 1)], d_a, n2, m2))
    assert len({pa.transform_len(it[3], it[4]) for it in items}) == 1
    return items


def expected(items):
    return [oracle.toeplitz_hash(k, n, s, m) for k, s, _, n, m in items]


def test_mixed_shared_and_own_seeds_match_oracle():
    items = mixed_batch()
    want = expected(items)
    blocks = [(dev(k), n, ds, m, out_for(m)) for k, _, ds, n, m in items]
    pa.toeplitz_hash_batched(blocks)
    for i, b in enumerate(blocks):
        assert np.array_equal(host(b[4], b[3]), want[i]), i
    # the same blocks one per call
    for i, (dk, n, ds, m, _) in enumerate(blocks[:3] + blocks[12:14]):
        assert np.array_equal(host(pa.toeplitz_hash(dk, n, ds, m), m), (want[:3] + want[12:14])[i]), i


def test_many_blocks_on_one_seed_across_lengths():
    # 40 blocks on one seed buffer: 3 lengths, each with its own spectrum
    g = np.random.default_rng(124)
    seed_bits = 3_000_000
    seed = wl.random_bits(seed_bits, wl.rng(124, wl.ROLE_SEED, 0))
    ds = dev(seed)
    items = []
    for i, (n, m) in enumerate([(200_000, 50_000)] * 16 + [(1_500_000, 300_000)] * 16 + [(2_000_000, 600_000)] * 8):
        key = wl.random_bits(n, wl.rng(124, wl.ROLE_KEY, i))
        # every block of a length uses the seed's first n + m - 1 bits
        items.append((key, seed[: wl.words(n + m - 1)], ds, n, m))
    want = expected(items)
    blocks = [(dev(k), n, ds_, m, out_for(m)) for k, _, ds_, n, m in items]
    pa.toeplitz_hash_batched(blocks)
    for i, b in enumerate(blocks):
        assert np.array_equal(host(b[4], b[3]), want[i]), i
    del g


def test_modified_toeplitz_with_a_shared_v():
    n, m = 1_000_000, 250_000
    v = wl.random_bits(n - 1, wl.rng(125, wl.ROLE_SEED, 0))
    dv = dev(v)
    keys = [wl.random_bits(n, wl.rng(125, wl.ROLE_KEY, i)) for i in range(6)]
    want = [oracle.modified_toeplitz_hash(k, n, v, m) for k in keys]
    blocks = [(dev(k), n, dv, m, out_for(m)) for k in keys]
    pa.modified_toeplitz_hash_batched(blocks)
    for i, b in enumerate(blocks):
        assert np.array_equal(host(b[4], m), want[i]), i


def test_graph_with_shared_seeds_replays_and_updates():
    items = mixed_batch()
    want = expected(items)
    blocks = [(dev(k), n, ds, m, out_for(m)) for k, _, ds, n, m in items]
    with pa.BatchGraph(blocks) as g:
        for rep in range(3):
            for b in blocks:
                b[4].fill_(-1)
            g.launch()
            for i, b in enumerate(blocks):
                assert np.array_equal(host(b[4], b[3]), want[i]), (rep, i)
        # new keys with the same sharing layout: accepted, and correct
        keys2 = [wl.random_bits(n, wl.rng(126, wl.ROLE_KEY, i)) for i, (_, _, _, n, _) in enumerate(items)]
        blocks2 = [(dev(k2), n, ds, m, out_for(m)) for k2, (_, _, ds, n, m) in zip(keys2, items)]
        torch.cuda.synchronize()
        g.update(blocks2)
        g.launch()
        for i, ((_, s, _, n, m), k2) in enumerate(zip(items, keys2)):
            assert np.array_equal(host(blocks2[i][4], m), oracle.toeplitz_hash(k2, n, s, m)), i
        # every block on its own seed: another layout, refused
        own = [(b[0], b[1], dev(wl.random_bits(b[1] + b[3] - 1, wl.rng(127, wl.ROLE_SEED, i))), b[3], b[4])
               for i, b in enumerate(blocks)]
        with pytest.raises(pa.PAError):
            g.update(own)
