"""pa_toeplitz_hash_noalloc (static device scratch, no allocation) against
pa_toeplitz_hash and the CPU oracle, bit for bit, over consecutive calls
of shrinking size: the largest block its scratch holds (transform length
27 * 2^19), then n = 10^6, then a ragged small block.  Each call must not
see anything of the previous call's contents in the shared scratch."""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def test_noalloc_matches_the_allocating_call_on_shrinking_inputs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    shapes = [(12_800_000, 1_280_000), (1_000_000, 250_000), (300_001, 70_003)]
    assert pa.transform_len(*shapes[0]) * 8 == pa.NOALLOC_SCRATCH_BYTES
    for i, (n, m) in enumerate(shapes):
        key, seed = wl.key_and_seed(40, n, m, i)
        dk, ds = dev(key), dev(seed)
        ref = pa.toeplitz_hash(dk, n, ds, m)  # also builds the transform tables of this length
        out = torch.full((wl.words(m),), -1, dtype=torch.int64, device="cuda")
        pa.toeplitz_hash_noalloc(dk, n, ds, m, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref.cpu().numpy().view(np.uint64)[: wl.words(m)]), (n, m)
        assert np.array_equal(got, oracle.toeplitz_hash(key, n, seed, m)), (n, m)
