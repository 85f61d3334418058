"""Parity at the sizes and launch configurations bench.py times: 256 blocks
of the n = 10^6, m = 250,000 workload in one batched call (default split and
the split the autotuner picks for batches), and the uneven 256-block batch
(n log-uniform in [2^18, 2^22]) with its graph replays.  Every block of
every batch is compared word for word with the CPU oracle; the oracle
outputs are computed once per module and reused for each launch form."""
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


@pytest.fixture(scope="module")
def uniform_batch():
    host_inputs = [wl.key_and_seed(4, N, M, i) + (N, M) for i in range(256)]
    refs = [oracle.toeplitz_hash(k, n, s, m) for k, s, n, m in host_inputs]
    return host_inputs, refs


@pytest.fixture(scope="module")
def uneven_batch():
    shapes = wl.batched_shapes(256, 4)
    host_inputs = [wl.key_and_seed(8, sh.n, sh.m, i) + (sh.n, sh.m) for i, sh in enumerate(shapes)]
    refs = [oracle.toeplitz_hash(k, n, s, m) for k, s, n, m in host_inputs]
    return host_inputs, refs


def _device_blocks(host_inputs):
    return [(dev(k), n, dev(s), m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda"))
            for k, s, n, m in host_inputs]


def _check_all(blocks, refs, what):
    torch.cuda.synchronize()
    bad = []
    for i, ((_, n, _, m, out), ref) in enumerate(zip(blocks, refs)):
        got = out.cpu().numpy().view(np.uint64)[: wl.words(m)]
        if not np.array_equal(got, ref):
            bad.append((i, n, m, int(np.sum(got != ref))))
    assert not bad, "%s: blocks differing from the oracle (index, n, m, words): %s" % (what, bad[:8])


@pytest.mark.parametrize("split", [(0, 0), (8, 64)])
def test_batched_256_finite_size_blocks(split, uniform_batch):
    host_inputs, refs = uniform_batch
    L = pa.transform_len(N, M)
    pa.tune_set(L, 1, *split)
    blocks = _device_blocks(host_inputs)
    pa.toeplitz_hash_batched(blocks)
    _check_all(blocks, refs, "batched split %s" % (split,))


def test_uneven_256_batch_and_its_graph(uneven_batch):
    host_inputs, refs = uneven_batch
    assert len({pa.transform_len(n, m) for _, _, n, m in host_inputs}) >= 10
    blocks = _device_blocks(host_inputs)
    pa.toeplitz_hash_batched(blocks)
    _check_all(blocks, refs, "eager batched call")
    for b in blocks:
        b[4].fill_(-1)
    with pa.BatchGraph(blocks) as g:
        for rep in range(3):
            g.launch()
            _check_all(blocks, refs, "graph replay %d" % rep)
            for b in blocks:
                b[4].fill_(-1)
            torch.cuda.synchronize()
