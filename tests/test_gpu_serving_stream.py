"""The serving workload at full scale: the 10,000-request stream (n
log-uniform in [1e5, 1e7], m/n uniform in [0.1, 0.5], 16 resident seeds of
2^24 bits, keys drawn from a pool of 64 device buffers of 10^7 bits) is
served under the same budget and limits bench.py uses.  Every served result
is compared with the same request run alone through pa_toeplitz_hash, and
a seeded sample of 64 requests plus every request with n <= 3e5 is compared
word for word with the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_SEEDS, SEED_BITS, POOL, POOL_BITS = 16, 1 << 24, 64, 10_000_000


def test_serving_stream_matches_alone_and_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    seeds = [wl.random_bits(SEED_BITS, wl.rng(5, wl.ROLE_SEED, i)) for i in range(N_SEEDS)]
    pool = [wl.random_bits(POOL_BITS, wl.rng(5, wl.ROLE_KEY, i)) for i in range(POOL)]
    dseeds = [torch.from_numpy(s.view(np.int64)).cuda() for s in seeds]
    dpool = [torch.from_numpy(k.view(np.int64)).cuda() for k in pool]
    reqs = wl.serving_requests(10_000, rate_per_s=1.0, n_seeds=N_SEEDS)
    offs, tot = [], 0
    for r in reqs:
        offs.append(tot)
        tot += wl.words(r.m)
    served = torch.zeros(tot, dtype=torch.int64, device="cuda")
    # the server's streams are not ordered after torch's: seeds, keys and the
    # zeroed outputs must be complete before the server reads or writes them
    torch.cuda.synchronize()
    with pa.Server(16 << 30, max_inflight=512, streams=4) as srv:
        ids = [srv.register_seed(d, SEED_BITS) for d in dseeds]
        for i, r in enumerate(reqs):
            srv.submit(ids[r.seed_id], dpool[i % POOL].data_ptr(), r.n, r.m, served.data_ptr() + 8 * offs[i])
        srv.drain()
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["peak_bytes_in_flight"] <= 16 << 30
    assert st["peak_inflight"] >= 2
    alone = torch.zeros_like(served)
    for i, r in enumerate(reqs):
        pa.toeplitz_hash(dpool[i % POOL], r.n, dseeds[r.seed_id], r.m,
                         alone[offs[i]: offs[i] + wl.words(r.m)])
    torch.cuda.synchronize()
    served_h = served.cpu().numpy().view(np.uint64)
    alone_h = alone.cpu().numpy().view(np.uint64)
    differ = [i for i, r in enumerate(reqs)
              if not np.array_equal(served_h[offs[i]: offs[i] + wl.words(r.m)],
                                    alone_h[offs[i]: offs[i] + wl.words(r.m)])]
    assert not differ, "served results differing from the request run alone: %s" % differ[:10]
    sample = set(int(i) for i in np.random.default_rng(55).choice(len(reqs), 64, replace=False))
    sample |= {i for i, r in enumerate(reqs) if r.n <= 300_000}
    assert len(sample) > 1000 and max(reqs[i].n for i in sample) > 5_000_000
    bad = []
    for i in sorted(sample):
        r = reqs[i]
        want = oracle.toeplitz_hash(pool[i % POOL], r.n, seeds[r.seed_id], r.m)
        if not np.array_equal(served_h[offs[i]: offs[i] + want.size], want):
            bad.append((i, r.n, r.m))
    assert not bad, "served results differing from the oracle (index, n, m): %s" % bad[:10]
