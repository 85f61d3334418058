"""Parity at the sizes and launch configurations bench.py times: 256 blocks
of the n = 10^6, m = 250,000 workload in one batched call (default split and
the split the autotuner picks for batches), the uneven 256-block batch and
its graph replay.  Every block is compared with the same block hashed alone,
and a seeded sample of blocks with the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, M = 1_000_000, 250_000


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


@pytest.fixture(autouse=True, scope="module")
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    yield
    pa.tune_set(pa.transform_len(N, M), 1, 0, 0)


def _check(blocks, host_inputs, sample):
    torch.cuda.synchronize()
    for i, (key, n, seed, m, out) in enumerate(blocks):
        alone = pa.toeplitz_hash(key, n, seed, m)
        torch.cuda.synchronize()
        assert torch.equal(out[: wl.words(m)].cpu(), alone[: wl.words(m)].cpu()), i
    for i in sample:
        k, s, n, m = host_inputs[i]
        got = blocks[i][4].cpu().numpy().view(np.uint64)[: wl.words(m)]
        assert np.array_equal(got, oracle.toeplitz_hash(k, n, s, m)), i


@pytest.mark.parametrize("split", [(0, 0), (8, 64)])
def test_batched_256_finite_size_blocks(split):
    L = pa.transform_len(N, M)
    pa.tune_set(L, 1, *split)
    host_inputs, blocks = [], []
    for i in range(256):
        k, s = wl.key_and_seed(4, N, M, i)
        host_inputs.append((k, s, N, M))
        blocks.append((dev(k), N, dev(s), M, torch.zeros(wl.words(M), dtype=torch.int64, device="cuda")))
    pa.toeplitz_hash_batched(blocks)
    _check(blocks, host_inputs, sample=[0, 97, 255])


def test_uneven_256_batch_and_its_graph():
    shapes = wl.batched_shapes(256, 4)
    host_inputs, blocks = [], []
    for i, sh in enumerate(shapes):
        k, s = wl.key_and_seed(8, sh.n, sh.m, i)
        host_inputs.append((k, s, sh.n, sh.m))
        blocks.append((dev(k), sh.n, dev(s), sh.m, torch.zeros(wl.words(sh.m), dtype=torch.int64, device="cuda")))
    pa.toeplitz_hash_batched(blocks)
    small = [i for i, sh in enumerate(shapes) if sh.n * sh.m < 2e11]
    sample = list(np.random.default_rng(81).choice(small, 6, replace=False))
    _check(blocks, host_inputs, sample)
    for b in blocks:
        b[4].fill_(-1)
    with pa.BatchGraph(blocks) as g:
        for _ in range(2):
            g.launch()
    _check(blocks, host_inputs, sample[:2])
